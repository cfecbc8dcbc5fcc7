// C ABI runtime of the Cartesian form-factor engine: contexts, device memory
// under an HBM budget, argument validation and kernel orchestration.
// Declarations and contracts: include/scarff.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/scarff.h"
#include "engine.h"

namespace scff {
hipError_t launch_vtable(const VRowDev* rows, int nrows, int vstride, const int n[3],
                         const double qmin[3], const double dq[3], float2* V, hipStream_t st);
hipError_t launch_grid(int state_blocks, int precision, const float2* V, int vstride,
                       const int4* terms, const int* coff, const int* cnpp, int n_chunks,
                       const float* Tp, const uint32_t* tp_bf, const int n[3], int n_states,
                       float2* f, float* f2, hipStream_t st);
int vtable_stride(const int n[3]);
hipError_t launch_points(int state_blocks, const VRowDev* rows, const int4* terms, const int* coff,
                         const int* cnpp, int n_chunks, const float* Tp, const double* q, int nq,
                         int n_states, float2* f, float* f2, hipStream_t st);
}  // namespace scff

using namespace scff;

namespace {
thread_local std::string g_err;
}  // namespace

void scff::set_error(const std::string& msg) { g_err = msg; }

namespace {

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int ok() {
    g_err.clear();
    return SCFF_OK;
}

// One device allocation owned by a context.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct scff_ctx {
    int device = 0;
    size_t budget = 0;   // 0 = unlimited
    size_t used = 0;
    Basis basis;
    PairData pairs;
    bool have_mol = false;
    std::vector<double> T;
    int n_states = 0;
    bool have_T = false;
    double eps = 0.0, spin = 1.0;
    Packed packed;
    bool packed_valid = false;   // host packing matches molecule/T/options
    bool uploaded = false;       // device copies match `packed`
    DevBuf d_rows, d_terms, d_coff, d_cnpp, d_tp, d_tpbf, d_vtab, d_f, d_f2, d_q;
    int vtab_rows = 0, vtab_stride = 0;
};

namespace {

void dev_free(scff_ctx* c, DevBuf& b) {
    if (b.p) {
        (void)hipFree(b.p);
        c->used -= b.bytes;
    }
    b.p = nullptr;
    b.bytes = 0;
}

// Ensure `b` holds at least `bytes`; keeps the old buffer if large enough.
int dev_reserve(scff_ctx* c, DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (b.p && b.bytes >= bytes) return SCFF_OK;
    const size_t old = b.bytes;
    if (c->budget && c->used - old + bytes > c->budget)
        return fail(SCFF_ENOMEM, "HBM budget exceeded: need " + std::to_string(c->used - old + bytes) +
                                     " bytes, budget " + std::to_string(c->budget));
    dev_free(c, b);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(SCFF_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    b.p = p;
    b.bytes = bytes;
    c->used += bytes;
    return SCFF_OK;
}

int hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(SCFF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return SCFF_OK;
}

int upload(scff_ctx* c, DevBuf& b, const void* src, size_t bytes, hipStream_t st) {
    int rc = dev_reserve(c, b, bytes);
    if (rc) return rc;
    if (bytes) return hip_check(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, st), "upload");
    return SCFF_OK;
}

int ensure_packed(scff_ctx* c, hipStream_t st) {
    if (!c->have_mol) return fail(SCFF_ESTATE, "no molecule loaded");
    if (!c->have_T) return fail(SCFF_ESTATE, "no transitions loaded");
    if (!c->packed_valid) {
        Packed pk;
        std::string err = pack(c->basis, c->pairs, c->n_states, c->T.data(), c->eps, c->spin, pk);
        if (!err.empty()) return fail(SCFF_EINVAL, err);
        c->packed = std::move(pk);
        c->packed_valid = true;
        c->uploaded = false;
    }
    if (!c->uploaded) {
        const Packed& p = c->packed;
        int rc;
        if ((rc = upload(c, c->d_rows, p.rows.data(), p.rows.size() * sizeof(VRowDev), st))) return rc;
        if ((rc = upload(c, c->d_terms, p.terms.data(), p.terms.size() * sizeof(int), st))) return rc;
        if ((rc = upload(c, c->d_coff, p.chunk_off.data(), p.chunk_off.size() * sizeof(int), st))) return rc;
        if ((rc = upload(c, c->d_cnpp, p.chunk_npp.data(), p.chunk_npp.size() * sizeof(int), st))) return rc;
        if ((rc = upload(c, c->d_tp, p.tp.data(), p.tp.size() * sizeof(float), st))) return rc;
        // split-BF16 operand: per entry (hi | lo << 16)
        std::vector<uint32_t> bf(p.tp.size());
        for (size_t i = 0; i < bf.size(); ++i) bf[i] = (uint32_t)p.tp_hi[i] | ((uint32_t)p.tp_lo[i] << 16);
        if ((rc = upload(c, c->d_tpbf, bf.data(), bf.size() * sizeof(uint32_t), st))) return rc;
        // the host vectors above must stay alive until the copies finish
        if ((rc = hip_check(hipStreamSynchronize(st), "upload sync"))) return rc;
        c->uploaded = true;
    }
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
    const int nrows = (int)c->packed.rows.size();
    const int stride = vtable_stride(g->n);
    int rc = dev_reserve(c, c->d_vtab, (size_t)nrows * stride * sizeof(float2));
    if (rc) return rc;
    double dq[3];
    for (int a = 0; a < 3; ++a) dq[a] = g->n[a] > 1 ? (g->qmax[a] - g->qmin[a]) / (g->n[a] - 1) : 0.0;
    c->vtab_rows = nrows;
    c->vtab_stride = stride;
    return hip_check(launch_vtable((const VRowDev*)c->d_rows.p, nrows, stride, g->n, g->qmin, dq,
                                   (float2*)c->d_vtab.p, st),
                     "vtable kernel launch");
}

int set_device(scff_ctx* c) { return hip_check(hipSetDevice(c->device), "hipSetDevice"); }

}  // namespace

// Pack, upload and report the device bytes an evaluation on grid g will hold
// (pair data, 1D tables and host-output staging for f and |f|^2).
int scff::ctx_prepare(scff_ctx* c, const scff_grid* g, size_t* bytes_needed) {
    int rc = validate_grid(g);
    if (rc) return rc;
    if ((rc = set_device(c))) return rc;
    if ((rc = ensure_packed(c, nullptr))) return rc;
    const size_t npts = (size_t)g->n[0] * g->n[1] * g->n[2];
    const int stride = vtable_stride(g->n);
    *bytes_needed = c->used + c->packed.rows.size() * (size_t)stride * sizeof(float2) +
                    npts * (size_t)c->n_states * (sizeof(float2) + sizeof(float));
    return ok();
}

extern "C" {

const char* scff_version(void) { return "scarff-mi355x 0.1 (gfx950)"; }

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
    c->budget = hbm_budget_bytes;
    *out = c;
    return ok();
}

void scff_destroy(scff_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (DevBuf* b : {&c->d_rows, &c->d_terms, &c->d_coff, &c->d_cnpp, &c->d_tp, &c->d_tpbf,
                      &c->d_vtab, &c->d_f, &c->d_f2, &c->d_q})
        dev_free(c, *b);
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
    PairData pd;
    build_pairs(b, pd);
    if (c->have_T && b.nbf != c->basis.nbf) {
        c->have_T = false;
        c->T.clear();
    }
    c->basis = std::move(b);
    c->pairs = std::move(pd);
    c->have_mol = true;
    c->packed_valid = false;
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
    c->T.assign(T, T + n);
    c->n_states = n_states;
    c->have_T = true;
    c->packed_valid = false;
    return ok();
}

int scff_set_options(scff_ctx* c, double screen_eps, double spin_factor) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (!(screen_eps >= 0.0) || !std::isfinite(screen_eps) || screen_eps >= 1.0)
        return fail(SCFF_EINVAL, "screen_eps must be in [0, 1)");
    if (!std::isfinite(spin_factor)) return fail(SCFF_EINVAL, "spin_factor must be finite");
    if (screen_eps != c->eps || spin_factor != c->spin) c->packed_valid = false;
    c->eps = screen_eps;
    c->spin = spin_factor;
    return ok();
}

int scff_query(scff_ctx* c, scff_info* info) {
    if (!c || !info) return fail(SCFF_EINVAL, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->nbf = c->basis.nbf;
    info->n_shells = c->basis.n_shells;
    info->n_states = c->have_T ? c->n_states : 0;
    info->shell_pairs_total = c->pairs.shell_pairs;
    info->pairs_total = (long long)c->pairs.cps.size();
    info->prim_pairs_total = c->pairs.prim_pairs_total;
    if (c->have_mol && c->have_T && !c->packed_valid) {
        Packed pk;
        std::string err = pack(c->basis, c->pairs, c->n_states, c->T.data(), c->eps, c->spin, pk);
        if (!err.empty()) return fail(SCFF_EINVAL, err);
        c->packed = std::move(pk);
        c->packed_valid = true;
        c->uploaded = false;
    }
    if (c->packed_valid) {
        info->pairs_kept = c->packed.pairs_kept;
        info->prim_comp_pairs_kept = c->packed.terms_kept;
    }
    info->device_bytes = c->used;
    return ok();
}

int scff_eval_grid(scff_ctx* c, const scff_grid* g, int precision, float* f, float* f2,
                   int out_on_device, void* hip_stream) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    int rc = validate_grid(g);
    if (rc) return rc;
    if (precision != SCFF_FP32 && precision != SCFF_BF16X3) return fail(SCFF_EINVAL, "unknown precision");
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    if ((rc = ensure_packed(c, st))) return rc;
    const size_t npts = (size_t)g->n[0] * g->n[1] * g->n[2];
    const size_t nout = npts * (size_t)c->n_states;
    if ((rc = build_vtables(c, g, st))) return rc;
    float2* df = (float2*)f;
    float* df2 = f2;
    if (!out_on_device) {
        if (f && (rc = dev_reserve(c, c->d_f, nout * sizeof(float2)))) return rc;
        if (f2 && (rc = dev_reserve(c, c->d_f2, nout * sizeof(float)))) return rc;
        df = f ? (float2*)c->d_f.p : nullptr;
        df2 = f2 ? (float*)c->d_f2.p : nullptr;
    }
    const Packed& p = c->packed;
    rc = hip_check(launch_grid(p.state_blocks, precision, (const float2*)c->d_vtab.p, c->vtab_stride,
                               (const int4*)c->d_terms.p, (const int*)c->d_coff.p,
                               (const int*)c->d_cnpp.p, p.n_chunks, (const float*)c->d_tp.p,
                               (const uint32_t*)c->d_tpbf.p, g->n, c->n_states, df, df2, st),
                   "grid kernel launch");
    if (rc) return rc;
    if (!out_on_device) {
        if (f && (rc = hip_check(hipMemcpyAsync(f, df, nout * sizeof(float2), hipMemcpyDeviceToHost, st), "D2H f")))
            return rc;
        if (f2 && (rc = hip_check(hipMemcpyAsync(f2, df2, nout * sizeof(float), hipMemcpyDeviceToHost, st), "D2H f2")))
            return rc;
        if ((rc = hip_check(hipStreamSynchronize(st), "stream sync"))) return rc;
    }
    return ok();
}

int scff_eval_points(scff_ctx* c, int n_q, const double* q, int precision, float* f, float* f2,
                     int out_on_device, void* hip_stream) {
    if (!c) return fail(SCFF_EINVAL, "ctx is NULL");
    if (n_q < 1 || n_q > (1 << 24)) return fail(SCFF_EINVAL, "n_q must be in 1..2^24");
    if (!q) return fail(SCFF_EINVAL, "q is NULL");
    if (precision != SCFF_FP32 && precision != SCFF_BF16X3) return fail(SCFF_EINVAL, "unknown precision");
    for (int i = 0; i < 3 * n_q; ++i)
        if (!std::isfinite(q[i])) return fail(SCFF_EINVAL, "non-finite q");
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    if ((rc = ensure_packed(c, st))) return rc;
    if ((rc = upload(c, c->d_q, q, (size_t)n_q * 3 * sizeof(double), st))) return rc;
    const size_t nout = (size_t)n_q * c->n_states;
    float2* df = (float2*)f;
    float* df2 = f2;
    if (!out_on_device) {
        if (f && (rc = dev_reserve(c, c->d_f, nout * sizeof(float2)))) return rc;
        if (f2 && (rc = dev_reserve(c, c->d_f2, nout * sizeof(float)))) return rc;
        df = f ? (float2*)c->d_f.p : nullptr;
        df2 = f2 ? (float*)c->d_f2.p : nullptr;
    }
    const Packed& p = c->packed;
    rc = hip_check(launch_points(p.state_blocks, (const VRowDev*)c->d_rows.p, (const int4*)c->d_terms.p,
                                 (const int*)c->d_coff.p, (const int*)c->d_cnpp.p, p.n_chunks,
                                 (const float*)c->d_tp.p, (const double*)c->d_q.p, n_q, c->n_states,
                                 df, df2, st),
                   "points kernel launch");
    if (rc) return rc;
    if (!out_on_device) {
        if (f && (rc = hip_check(hipMemcpyAsync(f, df, nout * sizeof(float2), hipMemcpyDeviceToHost, st), "D2H f")))
            return rc;
        if (f2 && (rc = hip_check(hipMemcpyAsync(f2, df2, nout * sizeof(float), hipMemcpyDeviceToHost, st), "D2H f2")))
            return rc;
    }
    // the uploaded q must outlive the kernel; the caller's q is host memory we copied from
    if ((rc = hip_check(hipStreamSynchronize(st), "stream sync"))) return rc;
    return ok();
}

int scff_export_vtensors(scff_ctx* c, const scff_grid* g, long long* n_terms_out, float* vx,
                         float* vy, float* vz, float* tp) {
    if (!c || !n_terms_out) return fail(SCFF_EINVAL, "NULL argument");
    int rc = validate_grid(g);
    if (rc) return rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = nullptr;
    if ((rc = ensure_packed(c, st))) return rc;
    const Packed& p = c->packed;
    *n_terms_out = p.terms_kept;
    if (!vx && !vy && !vz && !tp) return ok();
    if ((rc = build_vtables(c, g, st))) return rc;
    std::vector<float2> V((size_t)c->vtab_rows * c->vtab_stride);
    if ((rc = hip_check(hipMemcpyAsync(V.data(), c->d_vtab.p, V.size() * sizeof(float2), hipMemcpyDeviceToHost, st),
                        "D2H vtab")))
        return rc;
    if ((rc = hip_check(hipStreamSynchronize(st), "stream sync"))) return rc;
    const int SW = kStateBlock * p.state_blocks;
    long long t = 0;
    float* outs[3] = {vx, vy, vz};
    for (int ch = 0; ch < p.n_chunks; ++ch) {
        const int npp = p.chunk_npp[ch];
        for (int j = 0; j < kChunk; ++j)
            for (int k = 0; k < npp; ++k) {
                const int* tr = &p.terms[4 * ((size_t)p.chunk_off[ch] + (size_t)j * npp + k)];
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
                    for (int s = 0; s < p.n_states; ++s)
                        tp[(size_t)s * p.terms_kept + t] = p.tp[(size_t)(ch * kChunk + j) * SW + s];
                ++t;
            }
    }
    return ok();
}

}  // extern "C"
