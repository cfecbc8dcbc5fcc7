// Internal declarations of the form-factor engine (host precompute, device
// kernels, runtime).  Not part of the public ABI; see include/scarff.h.
#pragma once

#include <array>
#include <cstddef>
#include <cstdint>
#include <functional>
#include <shared_mutex>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/scarff.h"

namespace scff {

// Maximum primitive-pair terms per (virtual) component pair.  A component
// pair with more terms is split into several virtual pairs that share its
// packed transition weight, so any contraction length is supported.
constexpr int kMaxTermsPerPair = 9;
// Component pairs per unit: the layout granule of packed weights and term
// slots, and one pair of MFMA k-steps (4 pairs each) of the grid kernel.
constexpr int kChunk = 8;
// The grid kernel stages whole chunks of consecutive units that share a term
// count npp: at most kMaxUnitsPerChunk units and kMaxChunkTerms terms.
constexpr int kMaxUnitsPerChunk = 4;
constexpr int kMaxChunkTerms = kChunk * kMaxTermsPerPair;   // 72
// The grid kernel may split a grid's chunk list into up to kMaxSplit ranges
// (one workgroup per tile and range, FP64 partial sums reduced afterwards)
// when the grid has too few tiles to fill the device.
constexpr int kMaxSplit = 8;
// The pair-sum buffer G of the separable-integral and dipole paths holds
// nv x ncomp pair sums followed by ns x ncomp x kSepParts slices of their
// transition-weighted reduction.
constexpr int kSepParts = 64;
struct ChunkSplit {
    int n;                   // number of ranges (1 = no split)
    int lo[kMaxSplit + 1];   // range j is chunks [lo[j], lo[j+1]); lo[0] = 0, lo[n] = n_chunks
};
// Everything the fused grid kernel needs for one evaluation (one request of
// a batch): the 1D tables, the term slots and chunk list, the packed
// weights, the grid and its tiling, the split of the chunk list and the
// outputs.  Filled on the host; the batch kernel reads it from device memory.
struct GridDesc {
    const float2* V;          // 1D tables [rows][vstride]
    int vstride, vrows;
    const int4* terms;        // term slots (row ids)
    const int4* chunks;       // chunk table (first unit, units, npp, first slot)
    ChunkSplit sp;
    const uint32_t* Tp;       // packed weights (FP32 bits or split-BF16 halves)
    int3 n, ntiles;           // grid points and tiles per axis
    int nx_eval, n_states;
    float2* f;                // outputs (NULL to skip), or
    float* f2;
    double2* partial;         // FP64 partial sums of a split (NULL: unsplit)
    long long part_stride;
};
// States per MFMA row block.
constexpr int kStateBlock = 16;
constexpr int kMaxStates = 32;
constexpr int kMaxPrim = 32;

// One 1D V-tensor row is a (primitive pair, axis, power pair) triple.  On a
// q value of its axis it evaluates
//   V(q) = exp(-q^2/(4p)) * exp(i q P) * sum_u e[u] (i q)^u ,
// where every q-independent factor of the pair (contraction coefficients,
// primitive normalisation on this axis, and on the x row the Gaussian
// product prefactor with (pi/p)^{3/2}) is folded into e[].
// Device copy of a row.  The 1D tables are built from it in FP64 and rounded
// once to FP32 (phase argument, range reduction, Gaussian and polynomial).
struct VRowDev {
    double P;
    double inv4p;    // 1/(4p)
    double e[5];
    int deg;
    int axis;
};

// A device allocation owned by a context.
struct DeviceBuffer {
    void* p = nullptr;
    size_t bytes = 0;
};

struct PrepShell {
    int atom, l, nprim, off;
};

// Host-side view of a loaded molecule: validated basis plus the integer
// tables that lay out rows, component pairs and terms (no arithmetic of the
// method beyond normalisation constants).
struct Basis {
    int n_atoms = 0, n_shells = 0, nbf = 0;
    std::vector<double> xyz;
    std::vector<int> sh_atom, sh_l, sh_nprim, sh_off, sh_bf0;
    std::vector<double> exps, coefs;
    std::vector<double> cnorm;   // contracted normalisation per AO
    std::vector<double> n1d;     // per primitive, 1D normalisation for powers 0..2
    bool normalise = true;
    // layout tables
    int n_sp = 0, n_cp = 0;
    long long n_rows = 0, n_terms = 0;
    std::vector<PrepShell> shells;
    std::vector<int> sp;          // 4 ints per shell pair: sA, sB, row_off, term_off
    std::vector<int> sp_cp;       // first component pair of each shell pair
    std::vector<int> cp_first;    // first term of each component pair
    std::vector<int> cp_nterms;   // primitive pairs of each component pair
};

// Device pointers the precompute reads.
struct PrepInputs {
    const PrepShell* shells;
    const int4* sp;
    const int* sp_cp;
    const int* bf0;
    const int* cp_first;
    const int* cp_nterms;
    const double* xyz;
    const double* exps;
    const double* coefs;
    const double* n1d;
    const double* cnorm;
    const double* T;
    int nbf, n_states, n_sp, n_cp;
    long long n_rows_all, n_terms_all;
    double eps, spin;
};

// Device buffers of the precompute; rows/slots/cnpp/coff/chunks/tp32/tpbf are
// what the evaluation kernels consume.  cnpp/coff are per unit (terms per
// pair, first slot); chunks holds (first unit, units) per grid-kernel chunk.
struct PrepWork {
    DeviceBuffer rows_all, rowsum, trow, tbound, wt, cpmn, tp64, bsum, part, small, nk, nv, vbase,
        tmp, key, val, vinfo, tmp2, cnpp, csize, coff, tmp3, slots, tp32, tpbf, row_used, newid, tmp4,
        rows, uhist, chunks,
        vcp;   // per packed pair: its component pair (index of tp64), -1 for padding
    std::vector<int> chunk_host;   // staging of the chunk table (kept until the next prep)
    // pinned host memory of the context (kPinnedBytes, or NULL if it could
    // not be allocated): small readbacks and the chunk table travel through
    // it by DMA; every use is complete before run_prep returns
    void* pinned = nullptr;
};

constexpr size_t kPinnedBytes = (size_t)4 << 20;
constexpr size_t kPinnedTables = 4096;   // byte offset of the chunk table / molecule upload

struct PrepResult {
    int n_vpairs = 0, n_units = 0, n_chunks = 0, n_rows = 0, state_blocks = 1;
    long long n_slots = 0, pairs_kept = 0, terms_kept = 0;
};

// ---- host side of the precompute (precompute.cpp) ----
std::string build_basis(Basis& b, int n_atoms, const double* xyz, int n_shells,
                        const int* shell_atom, const int* shell_l, const int* shell_nprim,
                        const double* exps, const double* coefs, int normalise);

// ---- device precompute (prep.hip) ----
hipError_t run_prep(const PrepInputs& in, PrepWork& w, PrepResult& res, hipStream_t st,
                    const std::function<hipError_t(DeviceBuffer&, size_t)>& alloc);

// ---- static scratch (scratch.hip) ----
// Bytes of the per-device scratch array of scff_eval_grid_noalloc.
constexpr size_t kScratchBytes = (size_t)256 << 20;
// Device address of this device's array (device current; resolved once).
hipError_t scratch_address(int device, void** ptr);

// ---- FFT method (fft.hip) ----
// Molecule tables the transition-density kernel reads (device pointers).
struct FftMol {
    const PrepShell* shells;
    const int* bf0;
    const double* xyz;
    const double* exps;
    const double* coefs;
    const double* n1d;
    const double* cnorm;
    int n_shells;
};
// LDS a density workgroup may hold (its AO block grows with the basis: up to
// 1232 functions; 64-point tiles up to 240 functions, 32-point tiles up to 496).
constexpr size_t kFftLdsBytes = (size_t)78 << 10;
// Column blocks of 16 points per density workgroup for nbf_pad basis rows
// (4, 2 or 1), 0 if the AO block does not fit lds_limit bytes of LDS.
int fft_density_cb(int nbf_pad, size_t lds_limit);
// precision: SCFF_FP32 (FP32 weights, Ap holds ns RB KS 64 floats) or
// SCFF_BF16X3 (split-BF16 weights of 4 functions per lane, ns RB RB 64 uint4:
// the same bytes).
hipError_t launch_fft_pack(int precision, const double* T, const double* cnorm, int nbf, int ns, int RB, int KS,
                           double spin, void* Ap, hipStream_t st);
hipError_t launch_fft_density(int precision, const FftMol& m, const void* Ap, int nbf_pad, int ns, int RB, int KS,
                              const int n[3], const double x0[3], const double h[3], float* Z, float* phi,
                              double* psum, size_t lds_limit, long long* n_part, hipStream_t st);
hipError_t launch_fft_lines(float2* Z, int nb, const int n[3], hipStream_t st);
hipError_t launch_fft_finish(const float2* Z, const int n[3], int ns, double vpix, const double u[3], float2* f,
                             float* f2, double* psum, long long* n_part, hipStream_t st);
hipError_t launch_fft_sum(const double* part, int ns, long long n, double scale, double* out, int stride,
                          hipStream_t st);

// ---- spherical method (sph_tables.cpp, sph.hip) ----
// Polynomial degree of one geometry's D tensor (l_A + l_B <= 4 for d shells).
constexpr int kSphMaxN = 4;
// Gaunt entries per (lam mu, l m): L = |l - lam| + 2 j, j < 5.
constexpr int kSphGauntJ = 5;
constexpr int kSphMaxL = 48;   // largest lmax accepted
struct SphIndex {
    std::vector<std::array<int, 3>> nlm;   // (n, lam, mu) of the W tensor, n <= 4, lam = n, n-2, ...
    std::vector<std::array<int, 3>> uvw;   // monomial powers with u + v + w <= 4
};
SphIndex sph_index();
// Theta[uvw][nlm] complex (re, im), zero unless u + v + w = n.
std::vector<double> sph_theta_table(const SphIndex& ix);
// Gaunt[(lam mu)][(l m)][j], (lmax + 1)^2 harmonics l m, real.
std::vector<double> sph_gaunt_table(int lmax);
// One geometry (shell pair, primitive pair) of the spherical method.
struct SphGeom {
    int isp, pp;      // shell pair, primitive pair within it
    int ncp, npp;     // component pairs and primitive pairs of the shell pair
    int term0;        // first term of the shell pair
};
hipError_t launch_sph_geom(const SphGeom* geo, int n_geo, const VRowDev* rows, const int4* trow, const double* tp64,
                           int ns, const double2* theta, const int* uvw_idx, const int* nfirst, int n_nlm, int Lmax,
                           double4* gdat, double2* Yc, double2* W, hipStream_t st);
// Bq: workspace of nqb radii x ns 25 rows x n_geo double2 (the row operands
// of one batch of radii).
hipError_t launch_sph_q(const double4* gdat, const double2* Yc, const double2* W, int n_geo, int ns, int Lmax,
                        const int* nlm_of, const double* qs, int n_q, double* J, double2* Bq, int nqb, double2* Q,
                        hipStream_t st);
hipError_t launch_sph_couple(const double2* Q, const double* gaunt, int ns, int lmax, int Lmax, int n_q, double2* R,
                             hipStream_t st);
hipError_t launch_sph_grid(const double2* R, int ns, int lmax, int n_q, int n_theta, int n_phi, double2* F,
                           float2* f, float* f2, hipStream_t st);
hipError_t launch_sph_avg(const double2* R, int ns, int lmax, int n_q, double* avg, hipStream_t st);

// ---- runtime.cpp ----
// Gate between stream capture and device-wide runtime calls.  Allocation and
// release of device or pinned memory, event and stream creation and
// destruction, and device synchronisation take it shared; a thread that
// captures a stream into a graph holds it exclusively from the start to the
// end of the capture, so no such call (which the runtime may let touch or
// synchronise every stream, the capturing one included) runs meanwhile.
// Hold it only around the runtime call itself, never across another gated
// call.
std::shared_mutex& device_gate();
using GateShared = std::shared_lock<std::shared_mutex>;
// Thread-local message returned by scff_last_error().
void set_error(const std::string& msg);
// Pack and upload a context's problem for grid g on stream st and wait for
// it: when this returns, the precompute is complete in device memory, so an
// evaluation on any other stream may use it.  *bytes_needed receives the
// device bytes an evaluation on g in `precision` will hold in total.
int ctx_prepare(scff_ctx* c, const scff_grid* g, int precision, hipStream_t st, size_t* bytes_needed);
// Device bytes a context holds (its buffers are kept between calls).
size_t ctx_device_bytes(const scff_ctx* c);

// Two-phase evaluation of a prepared context for the server's batch runner:
// ctx_batch_reserve reserves every device buffer the evaluation needs (1D
// tables, device outputs, split partial sums) and fills the grid kernel's
// descriptor, without launching anything; ctx_batch_tables and
// ctx_batch_finish then only enqueue work (1D tables; split reduction and
// the copy of f / |f|^2 to host memory), so a batch's launches can be
// captured into a graph.
struct BatchEval {
    GridDesc desc;
    int cls = 0;               // grid kernel variant
    long long blocks = 0;      // tiles x splits of the evaluation
    int n_split = 1, nx_eval = 0;
    size_t nout = 0;           // output values (n_states x grid points)
};
int ctx_batch_reserve(scff_ctx* c, const scff_grid* g, int precision, bool want_f, bool want_f2, BatchEval* be);
int ctx_batch_tables(scff_ctx* c, const scff_grid* g, hipStream_t st);
int ctx_batch_finish(scff_ctx* c, const scff_grid* g, const BatchEval& be, float* host_f, float* host_f2,
                     hipStream_t st);
// After the batch's stream has been synchronised: the context has no
// asynchronous work pending.
void ctx_batch_done(scff_ctx* c);
// Grid kernel launchers (kernels.hip)
int grid_wg_per_cu(int state_blocks, int precision);
hipError_t launch_grid_batch(int cls, const GridDesc* descs, const int2* items, int n_items, int* counter, int wgs,
                             hipStream_t st);
hipError_t launch_zero_counters(int* c, int n, hipStream_t st);
int ctx_n_cu(const scff_ctx* c);

}  // namespace scff
