// C ABI runtime of the Cartesian form-factor engine: contexts, device memory
// under an HBM budget, argument validation and kernel orchestration.
// Declarations and contracts: include/scarff.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <utility>
#include <string>
#include <vector>

#include "../../include/scarff.h"
#include "engine.h"

namespace scff {
hipError_t launch_vtable(const VRowDev* rows, int nrows, int vstride, const int n[3],
                         const double qmin[3], const double dq[3], float2* V, hipStream_t st);
int vtable_stride(const int n[3]);
hipError_t launch_grid(int state_blocks, int precision, const float2* V, int vstride, int vrows,
                       const int4* terms, const int4* chunks, const ChunkSplit& sp, const float* Tp,
                       const uint32_t* tp_bf, const int n[3], int nx_eval, int n_states, float2* f, float* f2,
                       double2* part, hipStream_t st);
hipError_t launch_reduce(const double2* part, int n_split, const int n[3], int nx_eval, int n_states, float2* f,
                         float* f2, hipStream_t st);
hipError_t launch_mirror(const int n[3], int nx_eval, int n_states, float2* f, float* f2, hipStream_t st);
long long grid_tiles(int state_blocks, int precision, const int n[3], int nx_eval);
int grid_class(int state_blocks, int precision);
hipError_t grid_desc(int state_blocks, int precision, const float2* V, int vstride, int vrows, const int4* terms,
                     const int4* chunks, const ChunkSplit& sp, const float* Tp, const uint32_t* tp_bf,
                     const int n[3], int nx_eval, int n_states, float2* f, float* f2, double2* part, GridDesc* d,
                     long long* blocks);
hipError_t launch_points(int state_blocks, const VRowDev* rows, const int4* terms, const int* coff,
                         const int* cnpp, int n_chunks, const float* Tp, const double* q, int nq,
                         int n_states, float2* f, float* f2, hipStream_t st);
hipError_t launch_separable(const VRowDev* rows, int nrows, const int4* slots, const int* coff, const int* cnpp,
                            int n_units, const double* tp64, const int* vcp, int ns, const double2* w, const int n[3],
                            const double qmin[3], const double dq[3], double2* S, double2* G, double2* out,
                            hipStream_t st);
hipError_t launch_dipole(const VRowDev* rows, int nrows, const int4* slots, const int* coff, const int* cnpp,
                         int n_units, const double* tp64, const int* vcp, int ns, double2* S, double2* G,
                         double2* out, hipStream_t st);
hipError_t launch_points64(const VRowDev* rows, const int4* slots, const int* coff, const int* cnpp, int n_units,
                           const double* tp64, const int* vcp, int ns, const double* q, int nq, double* f2,
                           hipStream_t st);
}  // namespace scff

using namespace scff;

namespace {
thread_local std::string g_err;
}  // namespace

void scff::set_error(const std::string& msg) { g_err = msg; }

std::shared_mutex& scff::device_gate() {
    static std::shared_mutex m;
    return m;
}

// Timing events: precompute start/end, 1D tables start, grid kernel start/end.
// FFT method: packing start, density start, density end, transforms end.
// Spherical method: geometry kernel start, contraction start, contraction end, end.
enum { EV_PREP0, EV_PREP1, EV_VT0, EV_GRID0, EV_GRID1, EV_FFT0, EV_FFT1, EV_FFT2, EV_FFT3, EV_SPH0, EV_SPH1, EV_SPH2, EV_SPH3, EV_N };

struct scff_ctx {
    int device = 0;
    size_t budget = 0;   // 0 = unlimited
    size_t used = 0;
    Basis basis;
    bool have_mol = false;
    int n_states = 0;
    bool have_T = false;
    double eps = 0.0, spin = 1.0;
    // molecule tables on the device
    // molecule tables, uploaded together in one buffer: shells, shell pairs,
    // first component pair per shell pair, first basis function per shell,
    // first term / term count per component pair, positions, exponents,
    // coefficients, 1D primitive norms, contracted norms (byte offsets)
    DeviceBuffer d_mol, d_T;
    size_t mol_off[11] = {};
    std::vector<unsigned char> mol_stage;   // host staging of the upload
    // precompute results and evaluation buffers
    PrepWork prep;
    PrepResult pres;
    bool prepared = false;
    DeviceBuffer d_vtab, d_f, d_f2, d_q;
    int vtab_rows = 0, vtab_stride = 0;
    // timing
    bool timing = false;
    hipEvent_t ev[EV_N] = {};
    bool ev_recorded = false, ev_prep = false, fft_recorded = false, sph_recorded = false;
    // stream ordering: the end of the last asynchronous work on the context
    hipEvent_t order_ev = nullptr;
    hipStream_t order_st = nullptr;
    bool order_pending = false;
    // a call has enqueued device work that is not yet covered by order_ev
    // or a synchronisation (an error return in the middle of a call)
    bool async_open = false;
    int symmetry = 0;   // evaluate half of a grid symmetric about q = 0 (scff_set_symmetry)
    // check the precompute's tables on the host after every precompute
    // (environment SCFF_VALIDATE set and not "0" when the context is created)
    bool validate = false;
    int n_cu = 256;     // compute units of the device
    DeviceBuffer d_part;   // FP64 partial results of a split chunk list
    // FP64 low-momentum and separable work: weights / points, per-row and
    // per-pair values, per-state results
    DeviceBuffer d_lq_in, d_lq_S, d_lq_G, d_lq_out;
    // FFT method: packed weights, complex arrays of state pairs, partial
    // sums, Parseval sums, device copy of the density for host output
    DeviceBuffer d_fft_A, d_fft_Z, d_fft_part, d_fft_out, d_phi;
    // spherical method: constant tables (for sph_lmax), geometries, per-geometry
    // data, harmonics and W tensor, radii, contraction, R tensor, Legendre stage,
    // angular average
    DeviceBuffer d_sph_tab, d_sph_geo, d_sph_gdat, d_sph_Yc, d_sph_W, d_sph_B, d_sph_q, d_sph_Q, d_sph_R, d_sph_F, d_sph_avg,
        d_sph_J;
    int sph_lmax = -1;
    size_t sph_off[5] = {};   // theta, uvw index, nfirst, nlm_of, gaunt
    size_t lds_block = 65536;   // LDS bytes one workgroup may use
    void* scratch = nullptr;   // this device's static scratch array (scff_eval_grid_noalloc)
};

namespace {

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int ok() {
    g_err.clear();
    return SCFF_OK;
}

void dev_free(scff_ctx* c, DeviceBuffer& b) {
    if (b.p) {
        {
            GateShared g(device_gate());
            (void)hipFree(b.p);
        }
        c->used -= b.bytes;
    }
    b.p = nullptr;
    b.bytes = 0;
}

// Ensure `b` holds at least `bytes`; keeps the old buffer if large enough.
hipError_t dev_reserve_raw(scff_ctx* c, DeviceBuffer& b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (b.p && b.bytes >= bytes) return hipSuccess;
    const size_t old = b.bytes;
    if (c->budget && c->used - old + bytes > c->budget) return hipErrorOutOfMemory;
    dev_free(c, b);
    void* p = nullptr;
    hipError_t e;
    {
        GateShared g(device_gate());
        e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess) return e;
    b.p = p;
    b.bytes = bytes;
    c->used += bytes;
    return hipSuccess;
}

int dev_reserve(scff_ctx* c, DeviceBuffer& b, size_t bytes) {
    hipError_t e = dev_reserve_raw(c, b, bytes);
    if (e == hipErrorOutOfMemory)
        return fail(SCFF_ENOMEM, "HBM budget or device memory exceeded (need " + std::to_string(bytes) +
                                     " more bytes, context holds " + std::to_string(c->used) + ")");
    if (e != hipSuccess) return fail(SCFF_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
    return SCFF_OK;
}

int hip_check(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory) return fail(SCFF_ENOMEM, std::string(what) + ": out of device memory or HBM budget");
    if (e != hipSuccess) return fail(SCFF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return SCFF_OK;
}

int upload_sync(scff_ctx* c, DeviceBuffer& b, const void* src, size_t bytes) {
    int rc = dev_reserve(c, b, bytes);
    if (rc) return rc;
    if (bytes) {
        GateShared g(device_gate());
        return hip_check(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice), "upload");
    }
    return SCFF_OK;
}

int set_device(scff_ctx* c) { return hip_check(hipSetDevice(c->device), "hipSetDevice"); }

// A context may be driven from several streams in turn.  Work that depends on
// the context's device state (precompute results, tables, T) is ordered after
// the context's previous asynchronous work with an event, so a call on stream
// B never overtakes a call still running on stream A.
int order_after(scff_ctx* c, hipStream_t st) {
    c->async_open = true;
    if (!c->order_pending || st == c->order_st) return SCFF_OK;
    return hip_check(hipStreamWaitEvent(st, c->order_ev, 0), "stream ordering");
}
int order_mark(scff_ctx* c, hipStream_t st) {
    int rc;
    if (!c->order_ev) {
        GateShared g(device_gate());
        if ((rc = hip_check(hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming), "event create")))
            return rc;
    }
    if ((rc = hip_check(hipEventRecord(c->order_ev, st), "event record"))) return rc;
    c->order_st = st;
    c->order_pending = true;
    c->async_open = false;
    return SCFF_OK;
}
// host-side wait for the context's asynchronous work (before the host
// rewrites device buffers that it may still read)
int order_drain(scff_ctx* c) {
    if (!c->order_pending) return SCFF_OK;
    int rc = hip_check(hipEventSynchronize(c->order_ev), "event sync");
    if (rc == SCFF_OK) c->order_pending = false;
    return rc;
}
// st has been synchronised after order_after(c, st): everything is done
void order_done(scff_ctx* c) {
    c->order_pending = false;
    c->async_open = false;
}

int record(scff_ctx* c, int which, hipStream_t st) {
    if (!c->timing) return SCFF_OK;
    return hip_check(hipEventRecord(c->ev[which], st), "event record");
}

// Host check of the tables the grid kernel indexes with (on request): every
// term slot names a 1D-table row in [0, rows) and every chunk lies inside the
// unit and slot arrays.  A violation is an engine bug; it is reported as
// SCFF_EDEVICE before any kernel reads the tables.
int validate_prep(scff_ctx* c, hipStream_t st) {
    const PrepResult& p = c->pres;
    std::vector<int> slots((size_t)p.n_slots * 4);
    int rc;
    if (!slots.empty() &&
        (rc = hip_check(hipMemcpyAsync(slots.data(), c->prep.slots.p, slots.size() * sizeof(int),
                                       hipMemcpyDeviceToHost, st), "D2H slots")))
        return rc;
    if ((rc = hip_check(hipStreamSynchronize(st), "validation sync"))) return rc;
    for (size_t i = 0; i < slots.size(); i += 4)
        for (int a = 0; a < 3; ++a)
            if (slots[i + a] < 0 || slots[i + a] >= p.n_rows)
                return fail(SCFF_EDEVICE, "precompute produced a term slot outside the 1D tables (slot " +
                                              std::to_string(i / 4) + ", axis " + std::to_string(a) + ", row " +
                                              std::to_string(slots[i + a]) + " of " + std::to_string(p.n_rows) + ")");
    const std::vector<int>& ch = c->prep.chunk_host;
    if ((int)ch.size() < 4 * p.n_chunks) return fail(SCFF_EDEVICE, "chunk table shorter than its chunk count");
    for (int k = 0; k < p.n_chunks; ++k) {
        const long long u0 = ch[4 * k], nu = ch[4 * k + 1], npp = ch[4 * k + 2], s0 = ch[4 * k + 3];
        if (u0 < 0 || nu < 1 || nu > kMaxUnitsPerChunk || u0 + nu > p.n_units || npp < 1 ||
            npp > kMaxTermsPerPair || nu * kChunk * npp > kMaxChunkTerms || s0 < 0 ||
            s0 + nu * kChunk * npp > p.n_slots)
            return fail(SCFF_EDEVICE, "precompute produced a chunk outside the unit or slot arrays (chunk " +
                                          std::to_string(k) + ")");
    }
    return SCFF_OK;
}

int ensure_prepared(scff_ctx* c, hipStream_t st) {
    if (!c->have_mol) return fail(SCFF_ESTATE, "no molecule loaded");
    if (!c->have_T) return fail(SCFF_ESTATE, "no transitions loaded");
    if (c->prepared) return SCFF_OK;
    const Basis& b = c->basis;
    PrepInputs in{};
    const unsigned char* m = (const unsigned char*)c->d_mol.p;
    in.shells = (const PrepShell*)(m + c->mol_off[0]);
    in.sp = (const int4*)(m + c->mol_off[1]);
    in.sp_cp = (const int*)(m + c->mol_off[2]);
    in.bf0 = (const int*)(m + c->mol_off[3]);
    in.cp_first = (const int*)(m + c->mol_off[4]);
    in.cp_nterms = (const int*)(m + c->mol_off[5]);
    in.xyz = (const double*)(m + c->mol_off[6]);
    in.exps = (const double*)(m + c->mol_off[7]);
    in.coefs = (const double*)(m + c->mol_off[8]);
    in.n1d = (const double*)(m + c->mol_off[9]);
    in.cnorm = (const double*)(m + c->mol_off[10]);
    in.T = (const double*)c->d_T.p;
    in.nbf = b.nbf;
    in.n_states = c->n_states;
    in.n_sp = b.n_sp;
    in.n_cp = b.n_cp;
    in.n_rows_all = b.n_rows;
    in.n_terms_all = b.n_terms;
    in.eps = c->eps;
    in.spin = c->spin;
    PrepResult res;
    int rc;
    if ((rc = record(c, EV_PREP0, st))) return rc;
    hipError_t e = run_prep(in, c->prep, res, st, [c](DeviceBuffer& buf, size_t n) { return dev_reserve_raw(c, buf, n); });
    if (e != hipSuccess) return hip_check(e, "pair precompute");
    if ((rc = record(c, EV_PREP1, st))) return rc;
    c->ev_prep = c->timing;
    c->pres = res;
    if (c->validate && (rc = validate_prep(c, st))) return rc;
    c->prepared = true;
    return SCFF_OK;
}

int validate_grid(const scff_grid* g) {
    if (!g) return fail(SCFF_EINVAL, "grid is NULL");
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1 || g->n[a] > 4096) return fail(SCFF_EINVAL, "grid n must be in 1..4096");
        if (!std::isfinite(g->qmin[a]) || !std::isfinite(g->qmax[a]))
            return fail(SCFF_EINVAL, "grid bounds must be finite");
    }
    return SCFF_OK;
}

// 1D tables for the grid axes
int build_vtables(scff_ctx* c, const scff_grid* g, hipStream_t st) {
    const int nrows = c->pres.n_rows;
    const int stride = vtable_stride(g->n);
    // the grid kernel addresses the tables with 32-bit byte offsets
    if ((size_t)nrows * stride * sizeof(float2) > 0xffffffffull)
        return fail(SCFF_EINVAL, "1D tables of this grid exceed 4 GiB: evaluate it in slabs");
    int rc = dev_reserve(c, c->d_vtab, (size_t)nrows * stride * sizeof(float2));
    if (rc) return rc;
    double dq[3];
    for (int a = 0; a < 3; ++a) dq[a] = g->n[a] > 1 ? (g->qmax[a] - g->qmin[a]) / (g->n[a] - 1) : 0.0;
    c->vtab_rows = nrows;
    c->vtab_stride = stride;
    return hip_check(launch_vtable((const VRowDev*)c->prep.rows.p, nrows, stride, g->n, g->qmin, dq,
                                   (float2*)c->d_vtab.p, st),
                     "vtable kernel launch");
}

// every axis holds -q with q: index i and n-1-i are q and -q.  An axis of
// n > 1 points runs from -q_max to +q_max; a one-point axis holds the single
// value qmin (its qmax is not used), which is its own negative only at 0.
bool grid_symmetric(const scff_grid* g) {
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] == 1) {
            if (g->qmin[a] != 0.0) return false;
        } else if (g->qmin[a] != -g->qmax[a]) {
            return false;
        }
    }
    return true;
}

// How scff_eval_grid evaluates grid g: the planes it computes (ix < nx_eval;
// the rest are mirrored in the symmetric mode) and the split of the chunk
// list.  Every tile costs the same (it runs the whole chunk list), and the
// device holds two workgroups of 4 waves (or one of 8) per CU at once (the grid kernel's occupancy),
// so a launch of `tiles` workgroups takes ceil(tiles / slots) rounds: 64 or
// 1728 tiles on 512 slots leave most of one round idle.  Cutting the chunk
// list into S ranges of about equal work (a chunk costs units * (npp + 2):
// generator terms plus the contraction), one workgroup per tile and range,
// takes ceil(tiles * S / slots) rounds of 1/S the work; the FP64 partial sums
// are reduced afterwards (a pass over S x 16 bytes per output value, small
// next to the kernel).  S is the smallest value within 2 % of the best; a split
// must save at least 5 %, and its partial buffer is kept under
// kMaxPartBytes.  allow_split = false gives the unsplit plan.
constexpr size_t kMaxPartBytes = (size_t)1 << 30;

struct EvalPlan {
    int nx_eval;
    ChunkSplit sp;
};

EvalPlan plan_eval(const scff_ctx* c, const scff_grid* g, int precision, bool allow_split = true) {
    EvalPlan e{};
    e.nx_eval = (c->symmetry && grid_symmetric(g)) ? (g->n[0] + 1) / 2 : g->n[0];
    const int nch = c->pres.n_chunks;
    const long long tiles = grid_tiles(c->pres.state_blocks, precision, g->n, e.nx_eval);
    const long long slots = (long long)grid_wg_per_cu(c->pres.state_blocks, precision) * c->n_cu;
    const size_t part1 = (size_t)g->n[0] * g->n[1] * g->n[2] * (size_t)c->n_states * sizeof(double2);
    long long smax = std::min<long long>(kMaxSplit, nch);
    smax = std::min<long long>(smax, part1 ? (long long)(kMaxPartBytes / part1) : kMaxSplit);
    if (!allow_split) smax = 1;
    auto rounds_per_work = [&](long long S) { return (double)((tiles * S + slots - 1) / slots) / (double)S; };
    long long S = 1;
    double best = rounds_per_work(1);
    for (long long s2 = 2; s2 <= smax; ++s2) {
        const double r = rounds_per_work(s2);
        if (r < 0.98 * best) {
            best = r;
            S = s2;
        }
    }
    if (best > 0.95 * rounds_per_work(1)) S = 1;
    e.sp.n = (int)std::max<long long>(S, 1);
    const std::vector<int>& ch = c->prep.chunk_host;   // (first unit, units, npp, first slot) per chunk
    std::vector<double> pre(nch + 1, 0.0);
    for (int k = 0; k < nch; ++k) pre[k + 1] = pre[k] + (double)ch[4 * k + 1] * (ch[4 * k + 2] + 2.0);
    e.sp.lo[0] = 0;
    int k = 0;
    for (int j = 1; j < e.sp.n; ++j) {
        const double w = pre[nch] * j / e.sp.n;
        while (k < nch && pre[k] < w) ++k;
        e.sp.lo[j] = k;
    }
    e.sp.lo[e.sp.n] = nch;
    return e;
}

// The fused grid kernel (with the split reduction and the symmetric-mode
// mirror when the plan asks for them) on tables V, events around it.
int run_grid(scff_ctx* c, const scff_grid* g, int precision, const float2* V, int vstride, int vrows,
             const EvalPlan& pl, double2* part, float2* df, float* df2, hipStream_t st) {
    int rc;
    if ((rc = record(c, EV_GRID0, st))) return rc;
    const PrepResult& p = c->pres;
    // f(-q) = f(q)* for real T: on a grid symmetric about q = 0 the planes
    // ix >= ceil(nx/2) are the conjugates of computed ones (symmetric mode)
    rc = hip_check(launch_grid(p.state_blocks, precision, V, vstride, vrows, (const int4*)c->prep.slots.p,
                               (const int4*)c->prep.chunks.p, pl.sp, (const float*)c->prep.tp32.p,
                               (const uint32_t*)c->prep.tpbf.p, g->n, pl.nx_eval, c->n_states, df, df2, part, st),
                   "grid kernel launch");
    if (rc) return rc;
    if (pl.sp.n > 1 &&
        (rc = hip_check(launch_reduce(part, pl.sp.n, g->n, pl.nx_eval, c->n_states, df, df2, st), "reduce launch")))
        return rc;
    if (pl.nx_eval < g->n[0] &&
        (rc = hip_check(launch_mirror(g->n, pl.nx_eval, c->n_states, df, df2, st), "mirror kernel launch")))
        return rc;
    if ((rc = record(c, EV_GRID1, st))) return rc;
    c->ev_recorded = c->timing;
    return SCFF_OK;
}

int check_precision(int precision) {
    if (precision != SCFF_FP32 && precision != SCFF_BF16X3) return fail(SCFF_EINVAL, "unknown precision");
    return SCFF_OK;
}

void free_all(scff_ctx* c) {
    for (DeviceBuffer* b : {&c->d_mol, &c->d_T, &c->d_vtab, &c->d_part, &c->d_f, &c->d_f2, &c->d_q,
                            &c->d_lq_in, &c->d_lq_S, &c->d_lq_G, &c->d_lq_out, &c->d_fft_A, &c->d_fft_Z,
                            &c->d_fft_part, &c->d_fft_out, &c->d_phi, &c->d_sph_tab, &c->d_sph_geo,
                            &c->d_sph_gdat, &c->d_sph_Yc, &c->d_sph_W, &c->d_sph_B, &c->d_sph_q, &c->d_sph_Q, &c->d_sph_R,
                            &c->d_sph_F, &c->d_sph_avg, &c->d_sph_J})
        dev_free(c, *b);
    PrepWork& w = c->prep;
    for (DeviceBuffer* b : {&w.rows_all, &w.rowsum, &w.trow, &w.tbound, &w.wt, &w.cpmn, &w.tp64, &w.bsum,
                            &w.part, &w.small, &w.nk, &w.nv, &w.vbase, &w.tmp, &w.key, &w.val, &w.vinfo,
                            &w.tmp2, &w.cnpp, &w.csize, &w.coff, &w.tmp3, &w.slots, &w.tp32, &w.tpbf,
                            &w.row_used, &w.newid, &w.tmp4, &w.rows, &w.uhist, &w.chunks, &w.vcp})
        dev_free(c, *b);
}

int copy_out(const float2* df, float* f, const float* df2, float* f2, size_t nout, hipStream_t st) {
    int rc;
    if (f && (rc = hip_check(hipMemcpyAsync(f, df, nout * sizeof(float2), hipMemcpyDeviceToHost, st), "D2H f")))
        return rc;
    if (f2 && (rc = hip_check(hipMemcpyAsync(f2, df2, nout * sizeof(float), hipMemcpyDeviceToHost, st), "D2H f2")))
        return rc;
    return SCFF_OK;
}

}  // namespace

// Precompute a context's problem and report the device bytes an evaluation
// on g holds in total (precompute buffers, 1D tables, output staging).
int scff::ctx_prepare(scff_ctx* c, const scff_grid* g, int precision, hipStream_t st, size_t* bytes_needed) {
    int rc = validate_grid(g);
    if (rc) return rc;
    if ((rc = set_device(c))) return rc;
    if ((rc = order_after(c, st))) return rc;
    if ((rc = ensure_prepared(c, st))) return rc;
    // the last precompute kernels (row compaction, slot remap) are still in
    // flight on st: the caller evaluates on another stream, which is not
    // ordered after this one
    if ((rc = hip_check(hipStreamSynchronize(st), "precompute sync"))) return rc;
    order_done(c);
    const size_t npts = (size_t)g->n[0] * g->n[1] * g->n[2];
    const int stride = vtable_stride(g->n);
    // the 1D tables and output staging reuse buffers the context already
    // holds when those are large enough (a reused context)
    const size_t vt = (size_t)c->pres.n_rows * stride * sizeof(float2);
    const size_t of = npts * (size_t)c->n_states * sizeof(float2), of2 = npts * (size_t)c->n_states * sizeof(float);
    const EvalPlan pl = plan_eval(c, g, precision);
    const size_t op = pl.sp.n > 1 ? (size_t)pl.sp.n * npts * (size_t)c->n_states * sizeof(double2) : 0;
    const size_t held = c->d_vtab.bytes + c->d_f.bytes + c->d_f2.bytes + c->d_part.bytes;
    *bytes_needed = c->used - held + std::max(c->d_vtab.bytes, vt) + std::max(c->d_f.bytes, of) +
                    std::max(c->d_f2.bytes, of2) + std::max(c->d_part.bytes, op);
    return ok();
}

size_t scff::ctx_device_bytes(const scff_ctx* c) { return c ? c->used : 0; }

int scff::ctx_n_cu(const scff_ctx* c) { return c->n_cu; }

int scff::ctx_batch_reserve(scff_ctx* c, const scff_grid* g, int precision, bool want_f, bool want_f2,
                            BatchEval* be) {
    int rc = validate_grid(g);
    if (rc) return rc;
    if ((rc = check_precision(precision))) return rc;
    if (!c->prepared) return fail(SCFF_ESTATE, "batch evaluation of a context that is not prepared");
    if ((rc = set_device(c))) return rc;
    const size_t nout = (size_t)g->n[0] * g->n[1] * g->n[2] * (size_t)c->n_states;
    const int stride = vtable_stride(g->n);
    if ((size_t)c->pres.n_rows * stride * sizeof(float2) > 0xffffffffull)
        return fail(SCFF_EINVAL, "1D tables of this grid exceed 4 GiB: evaluate it in slabs");
    if ((rc = dev_reserve(c, c->d_vtab, (size_t)c->pres.n_rows * stride * sizeof(float2)))) return rc;
    if (want_f && (rc = dev_reserve(c, c->d_f, nout * sizeof(float2)))) return rc;
    if (want_f2 && (rc = dev_reserve(c, c->d_f2, nout * sizeof(float)))) return rc;
    EvalPlan pl = plan_eval(c, g, precision);
    double2* part = nullptr;
    if (pl.sp.n > 1) {
        if (dev_reserve(c, c->d_part, (size_t)pl.sp.n * nout * sizeof(double2)) == SCFF_OK)
            part = (double2*)c->d_part.p;
        else
            pl = plan_eval(c, g, precision, false);
    }
    const PrepResult& p = c->pres;
    hipError_t e = grid_desc(p.state_blocks, precision, (const float2*)c->d_vtab.p, stride, p.n_rows,
                             (const int4*)c->prep.slots.p, (const int4*)c->prep.chunks.p, pl.sp,
                             (const float*)c->prep.tp32.p, (const uint32_t*)c->prep.tpbf.p, g->n, pl.nx_eval,
                             c->n_states, want_f ? (float2*)c->d_f.p : nullptr, want_f2 ? (float*)c->d_f2.p : nullptr,
                             part, &be->desc, &be->blocks);
    if (e != hipSuccess) return hip_check(e, "grid descriptor");
    be->cls = grid_class(p.state_blocks, precision);
    be->n_split = pl.sp.n;
    be->nx_eval = pl.nx_eval;
    be->nout = nout;
    c->vtab_rows = p.n_rows;
    c->vtab_stride = stride;
    c->async_open = true;   // device work follows on the batch stream
    return ok();
}

int scff::ctx_batch_tables(scff_ctx* c, const scff_grid* g, hipStream_t st) {
    double dq[3];
    for (int a = 0; a < 3; ++a) dq[a] = g->n[a] > 1 ? (g->qmax[a] - g->qmin[a]) / (g->n[a] - 1) : 0.0;
    return hip_check(launch_vtable((const VRowDev*)c->prep.rows.p, c->vtab_rows, c->vtab_stride, g->n, g->qmin, dq,
                                   (float2*)c->d_vtab.p, st),
                     "vtable kernel launch");
}

int scff::ctx_batch_finish(scff_ctx* c, const scff_grid* g, const BatchEval& be, float* host_f, float* host_f2,
                           hipStream_t st) {
    int rc;
    float2* df = be.desc.partial ? (host_f ? (float2*)c->d_f.p : nullptr) : be.desc.f;
    float* df2 = be.desc.partial ? (host_f2 ? (float*)c->d_f2.p : nullptr) : be.desc.f2;
    if (be.n_split > 1 &&
        (rc = hip_check(launch_reduce(be.desc.partial, be.n_split, g->n, be.nx_eval, c->n_states, df, df2, st),
                        "reduce launch")))
        return rc;
    if (be.nx_eval < g->n[0] &&
        (rc = hip_check(launch_mirror(g->n, be.nx_eval, c->n_states, df, df2, st), "mirror kernel launch")))
        return rc;
    return copy_out(df, host_f, df2, host_f2, be.nout, st);
}

void scff::ctx_batch_done(scff_ctx* c) { order_done(c); }

extern "C" {

const char* scff_version(void) { return "scarff-mi355x 0.2 (gfx950)"; }

const char* scff_last_error(void) { return g_err.c_str(); }

int scff_create(int device, size_t hbm_budget_bytes, scff_ctx** out) {
    if (!out) return fail(SCFF_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(SCFF_EDEVICE, "no HIP device available");
    if (device < 0 || device >= n) return fail(SCFF_EINVAL, "device index out of range");
    if (hipSetDevice(device) != hipSuccess) return fail(SCFF_EDEVICE, "hipSetDevice failed");
    scff_ctx* c = new scff_ctx();
    c->device = device;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        c->n_cu = ncu;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        c->lds_block = (size_t)lds;
    // pinned staging of small readbacks and uploads; without it (allocation
    // refused) the same copies go through pageable memory
    GateShared g(device_gate());
    if (hipHostMalloc(&c->prep.pinned, kPinnedBytes, hipHostMallocDefault) != hipSuccess) c->prep.pinned = nullptr;
    c->budget = hbm_budget_bytes;
    const char* v = std::getenv("SCFF_VALIDATE");
    c->validate = v && v[0] && std::strcmp(v, "0") != 0;
    // resolved here, with the device current, so that the allocation-free
    // entry point does no set-up of its own; the ordering event likewise
    if (scratch_address(device, &c->scratch) != hipSuccess) c->scratch = nullptr;
    if (hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming) != hipSuccess) c->order_ev = nullptr;
    *out = c;
    return ok();
}

void scff_destroy(scff_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    // wait for this context's own device work only (other contexts keep
    // running); after a call that failed half-way, for the whole device
    if (c->async_open || order_drain(c) != SCFF_OK) {
        GateShared g(device_gate());
        (void)hipDeviceSynchronize();
    }
    free_all(c);
    {
        GateShared g(device_gate());
        for (hipEvent_t& e : c->ev)
            if (e) (void)hipEventDestroy(e);
        if (c->order_ev) (void)hipEventDestroy(c->order_ev);
        if (c->prep.pinned) (void)hipHostFree(c->prep.pinned);
    }
    delete c;
}

int scff_load_molecule(scff_ctx* c, int n_atoms, const double* xyz, int n_shells,
                       const int* shell_atom, const int* shell_l, const int* shell_nprim,
                       const double* exps, const double* coefs, int normalise, int* nbf_out) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    Basis b;
    std::string err = build_basis(b, n_atoms, xyz, n_shells, shell_atom, shell_l, shell_nprim, exps,
                                  coefs, normalise);
    if (!err.empty()) return fail(SCFF_EINVAL, err);
    int rc;
    if ((rc = set_device(c))) return rc;
    // upload the molecule tables (small host arrays).  Once the first table
    // is overwritten the previous molecule is gone: a failure past that point
    // leaves the context with no molecule (and no transitions) loaded.
    if ((rc = order_drain(c))) return rc;   // in-flight work may still read the old tables
    const bool had_T = c->have_T;
    const int old_nbf = c->basis.nbf;
    c->have_mol = false;
    c->have_T = false;
    c->prepared = false;
    {
        // one host staging buffer, one copy (each table at a 256-byte aligned offset)
        const std::pair<const void*, size_t> tabs[11] = {
            {b.shells.data(), b.shells.size() * sizeof(PrepShell)}, {b.sp.data(), b.sp.size() * sizeof(int)},
            {b.sp_cp.data(), b.sp_cp.size() * sizeof(int)},         {b.sh_bf0.data(), b.sh_bf0.size() * sizeof(int)},
            {b.cp_first.data(), b.cp_first.size() * sizeof(int)},   {b.cp_nterms.data(), b.cp_nterms.size() * sizeof(int)},
            {b.xyz.data(), b.xyz.size() * sizeof(double)},          {b.exps.data(), b.exps.size() * sizeof(double)},
            {b.coefs.data(), b.coefs.size() * sizeof(double)},      {b.n1d.data(), b.n1d.size() * sizeof(double)},
            {b.cnorm.data(), b.cnorm.size() * sizeof(double)}};
        size_t total = 0;
        for (int i = 0; i < 11; ++i) {
            c->mol_off[i] = total;
            total += (tabs[i].second + 255) & ~(size_t)255;
        }
        // pinned when it fits (the upload is synchronous, so the memory is free
        // again when it returns), else a pageable staging vector
        unsigned char* stage;
        if (c->prep.pinned && total <= kPinnedBytes - kPinnedTables) {
            stage = (unsigned char*)c->prep.pinned + kPinnedTables;
        } else {
            c->mol_stage.resize(total);
            stage = c->mol_stage.data();
        }
        std::memset(stage, 0, total);
        for (int i = 0; i < 11; ++i)
            if (tabs[i].second) std::memcpy(stage + c->mol_off[i], tabs[i].first, tabs[i].second);
        if ((rc = upload_sync(c, c->d_mol, stage, total))) return rc;
    }
    c->have_T = had_T && b.nbf == old_nbf;   // T (untouched) still matches the basis size
    c->basis = std::move(b);
    c->have_mol = true;
    if (nbf_out) *nbf_out = c->basis.nbf;
    return ok();
}

int scff_load_transitions(scff_ctx* c, int n_states, const double* T) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (!c->have_mol) return fail(SCFF_ESTATE, "load a molecule before its transitions");
    if (n_states < 1 || n_states > kMaxStates) return fail(SCFF_EINVAL, "n_states must be in 1..32");
    if (!T) return fail(SCFF_EINVAL, "T is NULL");
    const size_t n = (size_t)n_states * c->basis.nbf * c->basis.nbf;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(T[i])) return fail(SCFF_EINVAL, "non-finite entry in T");
    int rc;
    if ((rc = set_device(c))) return rc;
    if ((rc = order_drain(c))) return rc;   // in-flight work may still read the old T
    if ((rc = upload_sync(c, c->d_T, T, n * sizeof(double)))) return rc;
    c->n_states = n_states;
    c->have_T = true;
    c->prepared = false;
    return ok();
}

int scff_load_transitions_device(scff_ctx* c, int n_states, const double* T_dev, void* hip_stream) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (!c->have_mol) return fail(SCFF_ESTATE, "load a molecule before its transitions");
    if (n_states < 1 || n_states > kMaxStates) return fail(SCFF_EINVAL, "n_states must be in 1..32");
    if (!T_dev) return fail(SCFF_EINVAL, "T is NULL");
    int rc;
    if ((rc = set_device(c))) return rc;
    const size_t n = (size_t)n_states * c->basis.nbf * c->basis.nbf;
    hipStream_t st = (hipStream_t)hip_stream;
    if ((rc = order_after(c, st))) return rc;
    if ((rc = dev_reserve(c, c->d_T, n * sizeof(double)))) return rc;
    if ((rc = hip_check(hipMemcpyAsync(c->d_T.p, T_dev, n * sizeof(double), hipMemcpyDeviceToDevice, st),
                        "device copy of T")))
        return rc;
    if ((rc = order_mark(c, st))) return rc;
    c->n_states = n_states;
    c->have_T = true;
    c->prepared = false;
    return ok();
}

int scff_set_options(scff_ctx* c, double screen_eps, double spin_factor) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (!(screen_eps >= 0.0) || !std::isfinite(screen_eps) || screen_eps >= 1.0)
        return fail(SCFF_EINVAL, "screen_eps must be in [0, 1)");
    if (!std::isfinite(spin_factor)) return fail(SCFF_EINVAL, "spin_factor must be finite");
    if (screen_eps != c->eps || spin_factor != c->spin) c->prepared = false;
    c->eps = screen_eps;
    c->spin = spin_factor;
    return ok();
}

int scff_query(scff_ctx* c, scff_info* info) {
    if (!c || !info) return fail(SCFF_EINVAL, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    const Basis& b = c->basis;
    info->nbf = b.nbf;
    info->n_shells = b.n_shells;
    info->n_states = c->have_T ? c->n_states : 0;
    info->shell_pairs_total = b.n_sp;
    info->pairs_total = b.n_cp;
    info->prim_pairs_total = b.n_terms;
    if (c->have_mol && c->have_T) {
        int rc;
        if ((rc = set_device(c))) return rc;
        if (!c->prepared) {
            if ((rc = order_after(c, nullptr))) return rc;
            if ((rc = ensure_prepared(c, nullptr))) return rc;
            if ((rc = hip_check(hipStreamSynchronize(nullptr), "precompute sync"))) return rc;
            order_done(c);
        }
        info->pairs_kept = c->pres.pairs_kept;
        info->prim_comp_pairs_kept = c->pres.terms_kept;
        info->work_chunks = c->pres.n_chunks;
        info->work_units = c->pres.n_units;
    }
    info->device_bytes = c->used;
    return ok();
}

int scff_eval_grid(scff_ctx* c, const scff_grid* g, int precision, float* f, float* f2,
                   int out_on_device, void* hip_stream) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    int rc = validate_grid(g);
    if (rc) return rc;
    if ((rc = check_precision(precision))) return rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    c->ev_prep = false;
    if ((rc = order_after(c, st))) return rc;
    if ((rc = ensure_prepared(c, st))) return rc;
    const size_t npts = (size_t)g->n[0] * g->n[1] * g->n[2];
    const size_t nout = npts * (size_t)c->n_states;
    float2* df = (float2*)f;
    float* df2 = f2;
    if (!out_on_device) {
        if (f && (rc = dev_reserve(c, c->d_f, nout * sizeof(float2)))) return rc;
        if (f2 && (rc = dev_reserve(c, c->d_f2, nout * sizeof(float)))) return rc;
        df = f ? (float2*)c->d_f.p : nullptr;
        df2 = f2 ? (float*)c->d_f2.p : nullptr;
    }
    if ((rc = record(c, EV_VT0, st))) return rc;
    if ((rc = build_vtables(c, g, st))) return rc;
    // the partial buffer is the last reservation: a split that the context's
    // HBM budget cannot hold falls back to the unsplit evaluation (the same
    // values up to the order of the FP64 sums)
    EvalPlan pl = plan_eval(c, g, precision);
    double2* part = nullptr;
    if (pl.sp.n > 1) {
        if (dev_reserve(c, c->d_part, (size_t)pl.sp.n * nout * sizeof(double2)) == SCFF_OK)
            part = (double2*)c->d_part.p;
        else
            pl = plan_eval(c, g, precision, false);
    }
    if ((rc = run_grid(c, g, precision, (const float2*)c->d_vtab.p, c->vtab_stride, c->vtab_rows, pl, part, df,
                       df2, st)))
        return rc;
    if (!out_on_device) {
        if ((rc = copy_out(df, f, df2, f2, nout, st))) return rc;
        if ((rc = hip_check(hipStreamSynchronize(st), "stream sync"))) return rc;
        order_done(c);
    } else if ((rc = order_mark(c, st))) {
        return rc;
    }
    return ok();
}

int scff_eval_grid_noalloc(scff_ctx* c, const scff_grid* g, int precision, float* f, float* f2, void* hip_stream) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    int rc = validate_grid(g);
    if (rc) return rc;
    if ((rc = check_precision(precision))) return rc;
    if (!c->have_mol) return fail(SCFF_ESTATE, "no molecule loaded");
    if (!c->have_T) return fail(SCFF_ESTATE, "no transitions loaded");
    if (!c->prepared)
        return fail(SCFF_ESTATE, "the precompute of the loaded problem has not run (call scff_query or an "
                                 "evaluation after the last load or option change)");
    if (!c->scratch || !c->order_ev) return fail(SCFF_EDEVICE, "static scratch of the device is not available");
    // 1D tables first, then (when they fit) the partial sums of a split
    const int stride = vtable_stride(g->n);
    const size_t vt = (size_t)c->pres.n_rows * stride * sizeof(float2);
    const size_t vt_al = (vt + 255) & ~(size_t)255;
    if (vt > kScratchBytes || vt > 0xffffffffull)
        return fail(SCFF_EINVAL, "1D tables of this grid need " + std::to_string(vt) + " bytes; the static scratch "
                                 "holds " + std::to_string(kScratchBytes) + " (use scff_eval_grid)");
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    c->ev_prep = false;
    if ((rc = order_after(c, st))) return rc;
    unsigned char* base = (unsigned char*)c->scratch;
    float2* V = (float2*)base;
    double dq[3];
    for (int a = 0; a < 3; ++a) dq[a] = g->n[a] > 1 ? (g->qmax[a] - g->qmin[a]) / (g->n[a] - 1) : 0.0;
    if ((rc = record(c, EV_VT0, st))) return rc;
    if ((rc = hip_check(launch_vtable((const VRowDev*)c->prep.rows.p, c->pres.n_rows, stride, g->n, g->qmin, dq, V,
                                      st),
                        "vtable kernel launch")))
        return rc;
    const size_t nout = (size_t)g->n[0] * g->n[1] * g->n[2] * (size_t)c->n_states;
    EvalPlan pl = plan_eval(c, g, precision);
    double2* part = nullptr;
    if (pl.sp.n > 1) {
        if (vt_al + (size_t)pl.sp.n * nout * sizeof(double2) <= kScratchBytes)
            part = (double2*)(base + vt_al);
        else
            pl = plan_eval(c, g, precision, false);
    }
    if ((rc = run_grid(c, g, precision, V, stride, c->pres.n_rows, pl, part, (float2*)f, f2, st))) return rc;
    if ((rc = order_mark(c, st))) return rc;
    return ok();
}

int scff_set_symmetry(scff_ctx* c, int enable) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (enable != 0 && enable != 1) return fail(SCFF_EINVAL, "enable must be 0 or 1");
    c->symmetry = enable;
    return ok();
}

int scff_set_timing(scff_ctx* c, int enable) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    int rc;
    if ((rc = set_device(c))) return rc;
    if (enable && !c->ev[0]) {
        GateShared g(device_gate());
        for (hipEvent_t& e : c->ev)
            if ((rc = hip_check(hipEventCreate(&e), "hipEventCreate"))) return rc;
    }
    c->timing = enable != 0;
    c->ev_recorded = false;
    c->fft_recorded = false;
    c->sph_recorded = false;
    return ok();
}

int scff_last_timing(scff_ctx* c, float* prep_ms, float* vtable_ms, float* grid_ms) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (!c->timing || !c->ev_recorded) return fail(SCFF_ESTATE, "no timed evaluation recorded");
    int rc;
    if ((rc = hip_check(hipEventSynchronize(c->ev[EV_GRID1]), "event sync"))) return rc;
    float a = 0.f, b = 0.f, p = 0.f;
    if (c->ev_prep && (rc = hip_check(hipEventElapsedTime(&p, c->ev[EV_PREP0], c->ev[EV_PREP1]), "elapsed")))
        return rc;
    if ((rc = hip_check(hipEventElapsedTime(&a, c->ev[EV_VT0], c->ev[EV_GRID0]), "elapsed"))) return rc;
    if ((rc = hip_check(hipEventElapsedTime(&b, c->ev[EV_GRID0], c->ev[EV_GRID1]), "elapsed"))) return rc;
    if (prep_ms) *prep_ms = c->ev_prep ? p : 0.0f;
    if (vtable_ms) *vtable_ms = a;
    if (grid_ms) *grid_ms = b;
    return ok();
}

int scff_last_sph_timing(scff_ctx* c, float* geom_ms, float* contraction_ms, float* rest_ms) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (!c->timing || !c->sph_recorded) return fail(SCFF_ESTATE, "no timed spherical evaluation recorded");
    int rc;
    if ((rc = hip_check(hipEventSynchronize(c->ev[EV_SPH3]), "event sync"))) return rc;
    float a = 0.f, b = 0.f, t = 0.f;
    if ((rc = hip_check(hipEventElapsedTime(&a, c->ev[EV_SPH0], c->ev[EV_SPH1]), "elapsed")) ||
        (rc = hip_check(hipEventElapsedTime(&b, c->ev[EV_SPH1], c->ev[EV_SPH2]), "elapsed")) ||
        (rc = hip_check(hipEventElapsedTime(&t, c->ev[EV_SPH2], c->ev[EV_SPH3]), "elapsed")))
        return rc;
    if (geom_ms) *geom_ms = a;
    if (contraction_ms) *contraction_ms = b;
    if (rest_ms) *rest_ms = t;
    return ok();
}

int scff_last_fft_timing(scff_ctx* c, float* pack_ms, float* density_ms, float* transform_ms) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (!c->timing || !c->fft_recorded) return fail(SCFF_ESTATE, "no timed FFT evaluation recorded");
    int rc;
    if ((rc = hip_check(hipEventSynchronize(c->ev[EV_FFT3]), "event sync"))) return rc;
    float a = 0.f, b = 0.f, t = 0.f;
    if ((rc = hip_check(hipEventElapsedTime(&a, c->ev[EV_FFT0], c->ev[EV_FFT1]), "elapsed")) ||
        (rc = hip_check(hipEventElapsedTime(&b, c->ev[EV_FFT1], c->ev[EV_FFT2]), "elapsed")) ||
        (rc = hip_check(hipEventElapsedTime(&t, c->ev[EV_FFT2], c->ev[EV_FFT3]), "elapsed")))
        return rc;
    if (pack_ms) *pack_ms = a;
    if (density_ms) *density_ms = b;
    if (transform_ms) *transform_ms = t;
    return ok();
}

int scff_eval_points(scff_ctx* c, int n_q, const double* q, int precision, float* f, float* f2,
                     int out_on_device, void* hip_stream) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (n_q < 1 || n_q > (1 << 24)) return fail(SCFF_EINVAL, "n_q must be in 1..2^24");
    if (!q) return fail(SCFF_EINVAL, "q is NULL");
    int rc;
    if ((rc = check_precision(precision))) return rc;
    // points run on the FP32 vector units only (no matrix-core contraction)
    if (precision != SCFF_FP32)
        return fail(SCFF_EINVAL, "scff_eval_points supports SCFF_FP32 only (the split-BF16 contraction is a "
                                 "grid-kernel path)");
    for (int i = 0; i < 3 * n_q; ++i)
        if (!std::isfinite(q[i])) return fail(SCFF_EINVAL, "non-finite q");
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    if ((rc = order_after(c, st))) return rc;
    if ((rc = ensure_prepared(c, st))) return rc;
    if ((rc = dev_reserve(c, c->d_q, (size_t)n_q * 3 * sizeof(double)))) return rc;
    if ((rc = hip_check(hipMemcpyAsync(c->d_q.p, q, (size_t)n_q * 3 * sizeof(double), hipMemcpyHostToDevice, st),
                        "upload q")))
        return rc;
    const size_t nout = (size_t)n_q * c->n_states;
    float2* df = (float2*)f;
    float* df2 = f2;
    if (!out_on_device) {
        if (f && (rc = dev_reserve(c, c->d_f, nout * sizeof(float2)))) return rc;
        if (f2 && (rc = dev_reserve(c, c->d_f2, nout * sizeof(float)))) return rc;
        df = f ? (float2*)c->d_f.p : nullptr;
        df2 = f2 ? (float*)c->d_f2.p : nullptr;
    }
    const PrepResult& p = c->pres;
    rc = hip_check(launch_points(p.state_blocks, (const VRowDev*)c->prep.rows.p, (const int4*)c->prep.slots.p,
                                 (const int*)c->prep.coff.p, (const int*)c->prep.cnpp.p, p.n_units,
                                 (const float*)c->prep.tp32.p, (const double*)c->d_q.p, n_q, c->n_states,
                                 df, df2, st),
                   "points kernel launch");
    if (rc) return rc;
    if (!out_on_device && (rc = copy_out(df, f, df2, f2, nout, st))) return rc;
    // the host q array was copied asynchronously: finish before returning
    if ((rc = hip_check(hipStreamSynchronize(st), "stream sync"))) return rc;
    order_done(c);
    return ok();
}

int scff_export_vtensors(scff_ctx* c, const scff_grid* g, long long* n_terms_out, float* vx,
                         float* vy, float* vz, float* tp) {
    if (!c || !n_terms_out) return fail(SCFF_EINVAL, "NULL argument");
    int rc = validate_grid(g);
    if (rc) return rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = nullptr;
    if ((rc = order_after(c, st))) return rc;
    if ((rc = ensure_prepared(c, st))) return rc;
    const PrepResult& p = c->pres;
    *n_terms_out = p.terms_kept;
    if (!vx && !vy && !vz && !tp) {
        if ((rc = hip_check(hipStreamSynchronize(st), "stream sync"))) return rc;
        order_done(c);
        return ok();
    }
    if ((rc = build_vtables(c, g, st))) return rc;
    const int SW = kStateBlock * p.state_blocks;
    std::vector<float2> V((size_t)c->vtab_rows * c->vtab_stride);
    std::vector<int> slots((size_t)p.n_slots * 4), coff(p.n_units), cnpp(p.n_units);
    std::vector<float> tp32((size_t)p.n_vpairs * SW);
    struct Cp {
        void* dst;
        const void* src;
        size_t n;
    } cps[] = {{V.data(), c->d_vtab.p, V.size() * sizeof(float2)},
               {slots.data(), c->prep.slots.p, slots.size() * sizeof(int)},
               {coff.data(), c->prep.coff.p, coff.size() * sizeof(int)},
               {cnpp.data(), c->prep.cnpp.p, cnpp.size() * sizeof(int)},
               {tp32.data(), c->prep.tp32.p, tp32.size() * sizeof(float)}};
    for (const Cp& x : cps)
        if ((rc = hip_check(hipMemcpyAsync(x.dst, x.src, x.n, hipMemcpyDeviceToHost, st), "D2H export"))) return rc;
    if ((rc = hip_check(hipStreamSynchronize(st), "stream sync"))) return rc;
    order_done(c);
    long long t = 0;
    float* outs[3] = {vx, vy, vz};
    for (int ch = 0; ch < p.n_units; ++ch) {
        const int npp = cnpp[ch];
        for (int j = 0; j < kChunk; ++j)
            for (int k = 0; k < npp; ++k) {
                const int* tr = &slots[4 * ((size_t)coff[ch] + (size_t)j * npp + k)];
                if (!tr[3]) continue;
                for (int a = 0; a < 3; ++a) {
                    if (!outs[a]) continue;
                    const int na = g->n[a];
                    for (int i = 0; i < na; ++i) {
                        const float2 v = V[(size_t)tr[a] * c->vtab_stride + i];
                        outs[a][((size_t)t * na + i) * 2] = v.x;
                        outs[a][((size_t)t * na + i) * 2 + 1] = v.y;
                    }
                }
                if (tp)
                    for (int s = 0; s < c->n_states; ++s)
                        tp[(size_t)s * p.terms_kept + t] = tp32[(size_t)(ch * kChunk + j) * SW + s];
                ++t;
            }
    }
    return ok();
}

namespace {

// Precompute on the default stream and wait (host-result calls).
int prepare_sync(scff_ctx* c) {
    int rc;
    if ((rc = set_device(c))) return rc;
    if ((rc = order_after(c, nullptr))) return rc;
    return ensure_prepared(c, nullptr);
}

int finish_sync(scff_ctx* c) {
    int rc = hip_check(hipStreamSynchronize(nullptr), "stream sync");
    if (rc == SCFF_OK) order_done(c);
    return rc;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on the
// three-term recurrence of the Legendre polynomials).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-15) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace

int scff_eval_fft(scff_ctx* c, const scff_fft_grid* g, int precision, float* f, float* f2, float* phi,
                  double* parseval, int out_on_device, void* hip_stream) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (!g) return fail(SCFF_EINVAL, "grid is NULL");
    if (precision != SCFF_FP32 && precision != SCFF_BF16X3)
        return fail(SCFF_EINVAL, "precision must be SCFF_FP32 or SCFF_BF16X3");
    for (int a = 0; a < 3; ++a) {
        const int na = g->n[a];
        if (na < 1 || na > 1024 || (na & (na - 1)))
            return fail(SCFF_EINVAL, "FFT grid sizes must be powers of two in 1..1024");
        if (!std::isfinite(g->xmin[a]) || !std::isfinite(g->L[a]) || !(g->L[a] > 0.0))
            return fail(SCFF_EINVAL, "FFT box corner must be finite and its lengths positive");
    }
    if (!f && !f2 && !phi && !parseval) return fail(SCFF_EINVAL, "no output requested");
    if (!c->have_mol) return fail(SCFF_ESTATE, "no molecule loaded");
    if (!c->have_T) return fail(SCFF_ESTATE, "no transitions loaded");
    const int nbf = c->basis.nbf, ns = c->n_states;
    const int nbf_pad = (nbf + 15) & ~15;
    const size_t lds_limit = std::min(c->lds_block, kFftLdsBytes);
    if (fft_density_cb(nbf_pad, lds_limit) == 0)
        return fail(SCFF_EINVAL, "basis too large for the FFT method's density tile (" + std::to_string(nbf) +
                                     " functions)");
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    if ((rc = order_after(c, st))) return rc;
    const int RB = nbf_pad / 16, KS = nbf_pad / 4, nb = (ns + 1) / 2;
    const long long npts = (long long)g->n[0] * g->n[1] * g->n[2];
    const size_t nout = (size_t)npts * ns;
    const long long part_d = (npts + 15) / 16, part_f = (npts + 63) / 64;
    // the density kernel loads A operands up to 15 k-steps of 4 bytes (FP32) or 7 function groups
    // of 16 bytes (split BF16) per lane past a row block (unused): slack of 32 x 64 floats covers both
    if ((rc = dev_reserve(c, c->d_fft_A, ((size_t)ns * RB * KS + 32) * 64 * sizeof(float))) ||
        (rc = dev_reserve(c, c->d_fft_Z, (size_t)nb * npts * sizeof(float2))))
        return rc;
    if (parseval &&
        ((rc = dev_reserve(c, c->d_fft_part, (size_t)ns * (size_t)std::max(part_d, part_f) * sizeof(double))) ||
         (rc = dev_reserve(c, c->d_fft_out, (size_t)ns * 2 * sizeof(double)))))
        return rc;
    float2* df = (float2*)f;
    float* df2 = f2;
    float* dphi = phi;
    if (!out_on_device) {
        if (f && (rc = dev_reserve(c, c->d_f, nout * sizeof(float2)))) return rc;
        if (f2 && (rc = dev_reserve(c, c->d_f2, nout * sizeof(float)))) return rc;
        if (phi && (rc = dev_reserve(c, c->d_phi, nout * sizeof(float)))) return rc;
        df = f ? (float2*)c->d_f.p : nullptr;
        df2 = f2 ? (float*)c->d_f2.p : nullptr;
        dphi = phi ? (float*)c->d_phi.p : nullptr;
    }
    const unsigned char* mb = (const unsigned char*)c->d_mol.p;
    FftMol m;
    m.shells = (const PrepShell*)(mb + c->mol_off[0]);
    m.bf0 = (const int*)(mb + c->mol_off[3]);
    m.xyz = (const double*)(mb + c->mol_off[6]);
    m.exps = (const double*)(mb + c->mol_off[7]);
    m.coefs = (const double*)(mb + c->mol_off[8]);
    m.n1d = (const double*)(mb + c->mol_off[9]);
    m.cnorm = (const double*)(mb + c->mol_off[10]);
    m.n_shells = c->basis.n_shells;
    double h[3], u[3], vpix = 1.0, dq3 = 1.0;
    for (int a = 0; a < 3; ++a) {
        h[a] = g->L[a] / g->n[a];
        u[a] = g->xmin[a] / g->L[a];
        vpix *= h[a];
        dq3 *= 2.0 * M_PI / g->L[a];
    }
    double* part = parseval ? (double*)c->d_fft_part.p : nullptr;
    double* pout = parseval ? (double*)c->d_fft_out.p : nullptr;
    long long np_d = 0, np_f = 0;
    c->fft_recorded = false;
    if ((rc = record(c, EV_FFT0, st))) return rc;
    if ((rc = hip_check(launch_fft_pack(precision, (const double*)c->d_T.p, m.cnorm, nbf, ns, RB, KS, c->spin,
                                       c->d_fft_A.p, st),
                        "FFT weight packing")) ||
        (rc = record(c, EV_FFT1, st)) ||
        (rc = hip_check(launch_fft_density(precision, m, c->d_fft_A.p, nbf_pad, ns, RB, KS, g->n, g->xmin, h,
                                           (float*)c->d_fft_Z.p, dphi, part, lds_limit, &np_d, st),
                        "transition density kernel")) ||
        (rc = record(c, EV_FFT2, st)))
        return rc;
    if (parseval && (rc = hip_check(launch_fft_sum(part, ns, np_d, vpix, pout, 2, st), "Parseval sum")))
        return rc;
    if (f || f2 || parseval) {
        if ((rc = hip_check(launch_fft_lines((float2*)c->d_fft_Z.p, nb, g->n, st), "FFT line kernels")) ||
            (rc = hip_check(launch_fft_finish((const float2*)c->d_fft_Z.p, g->n, ns, vpix, u, df, df2, part, &np_f,
                                              st),
                            "FFT finish kernel")))
            return rc;
        if (parseval &&
            (rc = hip_check(launch_fft_sum(part, ns, np_f, dq3 / (8.0 * M_PI * M_PI * M_PI), pout + 1, 2, st),
                            "Parseval sum")))
            return rc;
    }
    if ((rc = record(c, EV_FFT3, st))) return rc;
    c->fft_recorded = c->timing;
    if (!out_on_device) {
        if ((rc = copy_out(df, f, df2, f2, nout, st))) return rc;
        if (phi && (rc = hip_check(hipMemcpyAsync(phi, dphi, nout * sizeof(float), hipMemcpyDeviceToHost, st),
                                   "D2H phi")))
            return rc;
    }
    if (parseval &&
        (rc = hip_check(hipMemcpyAsync(parseval, pout, (size_t)ns * 2 * sizeof(double), hipMemcpyDeviceToHost, st),
                        "D2H Parseval sums")))
        return rc;
    if (!out_on_device || parseval) {
        if ((rc = hip_check(hipStreamSynchronize(st), "stream sync"))) return rc;
        order_done(c);
    } else if ((rc = order_mark(c, st))) {
        return rc;
    }
    return ok();
}

int scff_eval_spherical(scff_ctx* c, int lmax, int n_q, const double* q, int n_theta, int n_phi, double* R,
                        float* f, float* f2, double* avg, int out_on_device, void* hip_stream) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (lmax < 0 || lmax > kSphMaxL) return fail(SCFF_EINVAL, "lmax must be in 0..48");
    if (n_q < 1 || n_q > 4096 || !q) return fail(SCFF_EINVAL, "n_q must be in 1..4096 and q non-NULL");
    for (int i = 0; i < n_q; ++i)
        if (!std::isfinite(q[i]) || q[i] < 0.0) return fail(SCFF_EINVAL, "radii must be finite and >= 0");
    if ((f || f2) && (n_theta < 2 || n_theta > 4096 || n_phi < 1 || n_phi > 8192))
        return fail(SCFF_EINVAL, "the angular grid needs 2..4096 polar and 1..8192 azimuthal points");
    if (!R && !f && !f2 && !avg) return fail(SCFF_EINVAL, "no output requested");
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    if ((rc = order_after(c, st))) return rc;
    if ((rc = ensure_prepared(c, st))) return rc;
    const int ns = c->n_states, Lmax = lmax + kSphMaxN;
    const int nl = (lmax + 1) * (lmax + 1), nL = (Lmax + 1) * (Lmax + 1);
    // constant tables for this lmax
    const SphIndex ix = sph_index();
    const int n_nlm = (int)ix.nlm.size();
    if (c->sph_lmax != lmax) {
        const std::vector<double> th = sph_theta_table(ix);
        const std::vector<double> ga = sph_gaunt_table(lmax);
        std::vector<int> uvw_idx(125, -1), nfirst(kSphMaxN + 2, 0), nlm_of((kSphMaxN + 1) * 25, -1);
        for (size_t a = 0; a < ix.uvw.size(); ++a)
            uvw_idx[(ix.uvw[a][0] * (kSphMaxN + 1) + ix.uvw[a][1]) * (kSphMaxN + 1) + ix.uvw[a][2]] = (int)a;
        for (int b = 0; b < n_nlm; ++b) {
            const auto& e = ix.nlm[b];
            nlm_of[e[0] * 25 + e[1] * e[1] + e[1] + e[2]] = b;
            nfirst[e[0] + 1] = b + 1;
        }
        const size_t sz[5] = {th.size() * sizeof(double), uvw_idx.size() * sizeof(int), nfirst.size() * sizeof(int),
                              nlm_of.size() * sizeof(int), ga.size() * sizeof(double)};
        const void* src[5] = {th.data(), uvw_idx.data(), nfirst.data(), nlm_of.data(), ga.data()};
        size_t total = 0;
        for (int i = 0; i < 5; ++i) {
            c->sph_off[i] = total;
            total += (sz[i] + 255) & ~(size_t)255;
        }
        std::vector<unsigned char> stage(total, 0);
        for (int i = 0; i < 5; ++i) std::memcpy(stage.data() + c->sph_off[i], src[i], sz[i]);
        c->sph_lmax = -1;
        if ((rc = hip_check(hipStreamSynchronize(st), "stream sync"))) return rc;
        if ((rc = upload_sync(c, c->d_sph_tab, stage.data(), total))) return rc;
        c->sph_lmax = lmax;
    }
    // geometries: every primitive pair of every shell pair
    const Basis& b = c->basis;
    std::vector<SphGeom> geo;
    for (int isp = 0; isp < b.n_sp; ++isp) {
        const int sA = b.sp[4 * isp], sB = b.sp[4 * isp + 1], term0 = b.sp[4 * isp + 3];
        const int lA = b.sh_l[sA], lB = b.sh_l[sB];
        const int ncA = (lA + 1) * (lA + 2) / 2, ncB = (lB + 1) * (lB + 2) / 2;
        const int ncp = sA == sB ? ncA * (ncA + 1) / 2 : ncA * ncB;
        const int npp = b.sh_nprim[sA] * b.sh_nprim[sB];
        for (int pp = 0; pp < npp; ++pp) geo.push_back(SphGeom{isp, pp, ncp, npp, term0});
    }
    const int n_geo = (int)geo.size();
    const size_t nrows = (size_t)ns * 25;
    // row operands of the contraction for a batch of radii: all of them when
    // they fit 4 GiB (an eighth of a set HBM budget), else as many as fit (a
    // batch of few radii would leave part of the device idle)
    const size_t per_q = nrows * (size_t)std::max(n_geo, 1) * sizeof(double2);
    const size_t bcap = c->budget ? std::min((size_t)4 << 30, c->budget / 8) : (size_t)4 << 30;
    const int nqb = (int)std::max<size_t>(1, std::min<size_t>((size_t)n_q, bcap / per_q));
    if ((rc = dev_reserve(c, c->d_sph_geo, geo.size() * sizeof(SphGeom))) ||
        (rc = dev_reserve(c, c->d_sph_gdat, geo.size() * sizeof(double4))) ||
        (rc = dev_reserve(c, c->d_sph_Yc, (size_t)n_geo * nL * sizeof(double2))) ||
        (rc = dev_reserve(c, c->d_sph_W, (size_t)n_geo * n_nlm * ns * sizeof(double2))) ||
        (rc = dev_reserve(c, c->d_sph_B, (size_t)nqb * per_q)) ||
        (rc = dev_reserve(c, c->d_sph_q, (size_t)n_q * sizeof(double))) ||
        (rc = dev_reserve(c, c->d_sph_Q, (size_t)n_q * nrows * nL * sizeof(double2))) ||
        (rc = dev_reserve(c, c->d_sph_J, (size_t)n_q * (Lmax + 2) * n_geo * sizeof(double))) ||
        (rc = dev_reserve(c, c->d_sph_R, (size_t)ns * n_q * nl * sizeof(double2))))
        return rc;
    if ((f || f2) && (rc = dev_reserve(c, c->d_sph_F, (size_t)ns * n_q * n_theta * (2 * lmax + 1) * sizeof(double2))))
        return rc;
    if (avg && !out_on_device && (rc = dev_reserve(c, c->d_sph_avg, (size_t)ns * n_q * sizeof(double)))) return rc;
    const size_t nout = (size_t)ns * n_q * (size_t)(f || f2 ? n_theta : 0) * (size_t)(f || f2 ? n_phi : 0);
    float2* df = (float2*)f;
    float* df2 = f2;
    double2* dR = (double2*)c->d_sph_R.p;
    double* davg = avg;
    if (!out_on_device) {
        if (f && (rc = dev_reserve(c, c->d_f, nout * sizeof(float2)))) return rc;
        if (f2 && (rc = dev_reserve(c, c->d_f2, nout * sizeof(float)))) return rc;
        df = f ? (float2*)c->d_f.p : nullptr;
        df2 = f2 ? (float*)c->d_f2.p : nullptr;
        davg = avg ? (double*)c->d_sph_avg.p : nullptr;
    } else if (R) {
        dR = (double2*)R;
    }
    const unsigned char* tb = (const unsigned char*)c->d_sph_tab.p;
    c->sph_recorded = false;
    if ((rc = hip_check(hipMemcpyAsync(c->d_sph_geo.p, geo.data(), geo.size() * sizeof(SphGeom),
                                       hipMemcpyHostToDevice, st), "upload geometries")) ||
        (rc = hip_check(hipMemcpyAsync(c->d_sph_q.p, q, (size_t)n_q * sizeof(double), hipMemcpyHostToDevice, st),
                        "upload radii")))
        return rc;
    if ((rc = record(c, EV_SPH0, st))) return rc;
    if ((rc = hip_check(launch_sph_geom((const SphGeom*)c->d_sph_geo.p, n_geo, (const VRowDev*)c->prep.rows_all.p,
                                        (const int4*)c->prep.trow.p, (const double*)c->prep.tp64.p, ns,
                                        (const double2*)(tb + c->sph_off[0]), (const int*)(tb + c->sph_off[1]),
                                        (const int*)(tb + c->sph_off[2]), n_nlm, Lmax, (double4*)c->d_sph_gdat.p,
                                        (double2*)c->d_sph_Yc.p, (double2*)c->d_sph_W.p, st),
                        "spherical geometry kernel")) ||
        (rc = record(c, EV_SPH1, st)) ||
        (rc = hip_check(launch_sph_q((const double4*)c->d_sph_gdat.p, (const double2*)c->d_sph_Yc.p,
                                     (const double2*)c->d_sph_W.p, n_geo, ns, Lmax, (const int*)(tb + c->sph_off[3]),
                                     (const double*)c->d_sph_q.p, n_q, (double*)c->d_sph_J.p,
                                     (double2*)c->d_sph_B.p, nqb, (double2*)c->d_sph_Q.p, st),
                        "spherical contraction kernel")) ||
        (rc = record(c, EV_SPH2, st)) ||
        (rc = hip_check(launch_sph_couple((const double2*)c->d_sph_Q.p, (const double*)(tb + c->sph_off[4]), ns, lmax,
                                          Lmax, n_q, dR, st),
                        "spherical coupling kernel")))
        return rc;
    if (davg && (rc = hip_check(launch_sph_avg(dR, ns, lmax, n_q, davg, st), "angular average kernel"))) return rc;
    if ((f || f2) && (rc = hip_check(launch_sph_grid(dR, ns, lmax, n_q, n_theta, n_phi, (double2*)c->d_sph_F.p, df,
                                                     df2, st),
                                     "spherical grid kernels")))
        return rc;
    if ((rc = record(c, EV_SPH3, st))) return rc;
    c->sph_recorded = c->timing;
    if (!out_on_device) {
        if ((rc = copy_out(df, f, df2, f2, nout, st))) return rc;
        if (R && (rc = hip_check(hipMemcpyAsync(R, dR, (size_t)ns * n_q * nl * sizeof(double2), hipMemcpyDeviceToHost,
                                                st), "D2H R")))
            return rc;
        if (avg && (rc = hip_check(hipMemcpyAsync(avg, davg, (size_t)ns * n_q * sizeof(double), hipMemcpyDeviceToHost,
                                                  st), "D2H average")))
            return rc;
        if ((rc = hip_check(hipStreamSynchronize(st), "stream sync"))) return rc;
        order_done(c);
    } else {
        // host arrays (geometries, radii) were read by asynchronous copies: wait
        if ((rc = hip_check(hipStreamSynchronize(st), "stream sync"))) return rc;
        order_done(c);
    }
    return ok();
}

int scff_eval_separable(scff_ctx* c, const scff_grid* g, const double* wx, const double* wy, const double* wz,
                        double* out) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    int rc = validate_grid(g);
    if (rc) return rc;
    if (!wx || !wy || !wz || !out) return fail(SCFF_EINVAL, "weights and output must not be NULL");
    const double* ws[3] = {wx, wy, wz};
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i < 2 * g->n[a]; ++i)
            if (!std::isfinite(ws[a][i])) return fail(SCFF_EINVAL, "non-finite weight");
    if ((rc = prepare_sync(c))) return rc;
    const PrepResult& p = c->pres;
    const size_t nw = (size_t)g->n[0] + g->n[1] + g->n[2];
    const size_t nv = (size_t)p.n_units * kChunk;
    if ((rc = dev_reserve(c, c->d_lq_in, nw * sizeof(double2))) ||
        (rc = dev_reserve(c, c->d_lq_S, (size_t)p.n_rows * sizeof(double2))) ||
        (rc = dev_reserve(c, c->d_lq_G, (nv + (size_t)c->n_states * kSepParts) * sizeof(double2))) ||
        (rc = dev_reserve(c, c->d_lq_out, (size_t)c->n_states * sizeof(double2))))
        return rc;
    size_t off = 0;
    for (int a = 0; a < 3; ++a) {
        if ((rc = hip_check(hipMemcpyAsync((double2*)c->d_lq_in.p + off, ws[a], g->n[a] * sizeof(double2),
                                           hipMemcpyHostToDevice, nullptr),
                            "upload weights")))
            return rc;
        off += g->n[a];
    }
    double dq[3];
    for (int a = 0; a < 3; ++a) dq[a] = g->n[a] > 1 ? (g->qmax[a] - g->qmin[a]) / (g->n[a] - 1) : 0.0;
    if ((rc = hip_check(launch_separable((const VRowDev*)c->prep.rows.p, p.n_rows, (const int4*)c->prep.slots.p,
                                         (const int*)c->prep.coff.p, (const int*)c->prep.cnpp.p, p.n_units,
                                         (const double*)c->prep.tp64.p, (const int*)c->prep.vcp.p, c->n_states,
                                         (const double2*)c->d_lq_in.p, g->n, g->qmin, dq, (double2*)c->d_lq_S.p,
                                         (double2*)c->d_lq_G.p, (double2*)c->d_lq_out.p, nullptr),
                        "separable kernels")))
        return rc;
    if ((rc = hip_check(hipMemcpyAsync(out, c->d_lq_out.p, (size_t)c->n_states * sizeof(double2),
                                       hipMemcpyDeviceToHost, nullptr),
                        "D2H separable")))
        return rc;
    if ((rc = finish_sync(c))) return rc;
    return ok();
}

int scff_dipole(scff_ctx* c, const double* dE, double* mu, double* f0) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (!mu) return fail(SCFF_EINVAL, "mu must not be NULL");
    if (f0 && !dE) return fail(SCFF_EINVAL, "oscillator strengths need the transition energies dE");
    int rc;
    if ((rc = prepare_sync(c))) return rc;
    const PrepResult& p = c->pres;
    const int ns = c->n_states;
    if (dE)
        for (int s = 0; s < ns; ++s)
            if (!std::isfinite(dE[s])) return fail(SCFF_EINVAL, "non-finite transition energy");
    const size_t nv = (size_t)p.n_units * kChunk;
    if ((rc = dev_reserve(c, c->d_lq_S, (size_t)p.n_rows * sizeof(double2))) ||
        (rc = dev_reserve(c, c->d_lq_G, 4 * (nv + (size_t)ns * kSepParts) * sizeof(double2))) ||
        (rc = dev_reserve(c, c->d_lq_out, (size_t)ns * 4 * sizeof(double2))))
        return rc;
    if ((rc = hip_check(launch_dipole((const VRowDev*)c->prep.rows.p, p.n_rows, (const int4*)c->prep.slots.p,
                                      (const int*)c->prep.coff.p, (const int*)c->prep.cnpp.p, p.n_units,
                                      (const double*)c->prep.tp64.p, (const int*)c->prep.vcp.p, ns,
                                      (double2*)c->d_lq_S.p, (double2*)c->d_lq_G.p, (double2*)c->d_lq_out.p,
                                      nullptr),
                        "dipole kernels")))
        return rc;
    std::vector<double2> r((size_t)ns * 4);
    if ((rc = hip_check(hipMemcpyAsync(r.data(), c->d_lq_out.p, r.size() * sizeof(double2), hipMemcpyDeviceToHost,
                                       nullptr),
                        "D2H dipole")))
        return rc;
    if ((rc = finish_sync(c))) return rc;
    for (int s = 0; s < ns; ++s) {
        // f'(0) = i * (derivative / i): the imaginary part is the real sum
        double m2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            mu[3 * s + a] = r[4 * (size_t)s + 1 + a].x;
            m2 += mu[3 * s + a] * mu[3 * s + a];
        }
        if (f0) f0[s] = 2.0 / 3.0 * dE[s] * m2;
    }
    return ok();
}

int scff_dipole_fit(scff_ctx* c, double q_fit, const double* dE, double* coef, double* f0_fit) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (!coef) return fail(SCFF_EINVAL, "coef must not be NULL");
    if (!(q_fit > 0.0) || !std::isfinite(q_fit)) return fail(SCFF_EINVAL, "q_fit must be positive and finite");
    if (f0_fit && !dE) return fail(SCFF_EINVAL, "oscillator strengths need the transition energies dE");
    int rc;
    if ((rc = prepare_sync(c))) return rc;
    const PrepResult& p = c->pres;
    const int ns = c->n_states;
    // kFitShells radii q_k = q_fit k / kFitShells; on each, the product rule
    // of kFitTheta Gauss-Legendre nodes in cos(theta) and kFitPhi equally
    // spaced phi (exact for the sphere average of polynomials of degree < 12)
    constexpr int kFitShells = 8, kFitTheta = 6, kFitPhi = 12;
    std::vector<double> xt, wt;
    gauss_legendre(kFitTheta, xt, wt);
    const int ndir = kFitTheta * kFitPhi, nq = kFitShells * ndir;
    std::vector<double> q(3 * (size_t)nq), wdir(ndir);
    for (int k = 0; k < kFitShells; ++k) {
        const double r = q_fit * (k + 1) / kFitShells;
        for (int t = 0; t < kFitTheta; ++t)
            for (int ph = 0; ph < kFitPhi; ++ph) {
                const double ct = xt[t], st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
                const double phi = 2.0 * M_PI * ph / kFitPhi;
                const size_t i = (size_t)k * ndir + t * kFitPhi + ph;
                q[3 * i] = r * st * std::cos(phi);
                q[3 * i + 1] = r * st * std::sin(phi);
                q[3 * i + 2] = r * ct;
                wdir[t * kFitPhi + ph] = wt[t] / (2.0 * kFitPhi);
            }
    }
    if ((rc = dev_reserve(c, c->d_lq_in, q.size() * sizeof(double))) ||
        (rc = dev_reserve(c, c->d_lq_out, (size_t)ns * nq * sizeof(double))))
        return rc;
    if ((rc = hip_check(hipMemcpyAsync(c->d_lq_in.p, q.data(), q.size() * sizeof(double), hipMemcpyHostToDevice,
                                       nullptr),
                        "upload points")))
        return rc;
    if ((rc = hip_check(launch_points64((const VRowDev*)c->prep.rows.p, (const int4*)c->prep.slots.p,
                                        (const int*)c->prep.coff.p, (const int*)c->prep.cnpp.p, p.n_units,
                                        (const double*)c->prep.tp64.p, (const int*)c->prep.vcp.p, ns,
                                        (const double*)c->d_lq_in.p, nq, (double*)c->d_lq_out.p, nullptr),
                        "points64 kernel")))
        return rc;
    std::vector<double> f2((size_t)ns * nq);
    if ((rc = hip_check(hipMemcpyAsync(f2.data(), c->d_lq_out.p, f2.size() * sizeof(double), hipMemcpyDeviceToHost,
                                       nullptr),
                        "D2H |f|^2")))
        return rc;
    if ((rc = finish_sync(c))) return rc;
    for (int s = 0; s < ns; ++s) {
        // least squares of <|f|^2>(x) = a0 + a1 x + a2 x^2 in x = (q / q_fit)^2
        double M[3][3] = {}, v[3] = {};
        for (int k = 0; k < kFitShells; ++k) {
            double avg = 0.0;
            for (int d = 0; d < ndir; ++d) avg += wdir[d] * f2[(size_t)s * nq + (size_t)k * ndir + d];
            const double x = std::pow((k + 1.0) / kFitShells, 2), b[3] = {1.0, x, x * x};
            for (int i = 0; i < 3; ++i) {
                v[i] += b[i] * avg;
                for (int j = 0; j < 3; ++j) M[i][j] += b[i] * b[j];
            }
        }
        // Gaussian elimination with partial pivoting on the 3 x 3 normal equations
        int piv[3] = {0, 1, 2};
        for (int col = 0; col < 3; ++col) {
            int best = col;
            for (int r2 = col + 1; r2 < 3; ++r2)
                if (std::fabs(M[piv[r2]][col]) > std::fabs(M[piv[best]][col])) best = r2;
            std::swap(piv[col], piv[best]);
            for (int r2 = col + 1; r2 < 3; ++r2) {
                const double m = M[piv[r2]][col] / M[piv[col]][col];
                for (int j = col; j < 3; ++j) M[piv[r2]][j] -= m * M[piv[col]][j];
                v[piv[r2]] -= m * v[piv[col]];
            }
        }
        double a[3];
        for (int i = 2; i >= 0; --i) {
            double t = v[piv[i]];
            for (int j = i + 1; j < 3; ++j) t -= M[piv[i]][j] * a[j];
            a[i] = t / M[piv[i]][i];
        }
        coef[3 * s] = a[0];
        coef[3 * s + 1] = a[1] / (q_fit * q_fit);
        coef[3 * s + 2] = a[2] / (q_fit * q_fit * q_fit * q_fit);
        if (f0_fit) f0_fit[s] = 2.0 * dE[s] * coef[3 * s + 1];
    }
    return ok();
}

}  // extern "C"
