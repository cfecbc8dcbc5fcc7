// FP64 device kernels on the precompute's 1D V-tensor rows, with cost linear
// in the grid axes instead of their product (paper Sec. 5.3, separable
// integrals from the 1D V-tensors; Sec. 6, the low-momentum limit):
//
//  * separable integral  I_s = sum_{ix,iy,iz} wx[ix] wy[iy] wz[iz] f_s(q)
//      = sum_t Tp_s(t) (sum_ix wx V^x_t) (sum_iy wy V^y_t) (sum_iz wz V^z_t):
//    one weighted row sum per 1D row, then one complex triple product per
//    term, then the transition-weighted sum over packed pairs;
//  * transition dipole  mu_s = grad_q Im f_s at q = 0: each row's value and
//    first derivative at q = 0 are V(0) = e_0 and V'(0) = i (P e_0 + e_1), so
//    d f_s / d q_x (0) = i sum_t Tp_s(t) (P e_0 + e_1)^x e_0^y e_0^z;
//  * |f_s(q)|^2 at arbitrary points entirely in FP64 (rows evaluated on the
//    fly, FP64 transition weights), for the angular-average fit of Sec. 6.
//
// All sums run in FP64 with the FP64 packed weights tp64[component pair][s];
// the reductions over packed pairs use a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include "engine.h"
#include "vrow.h"

namespace scff {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// S[r] = sum_i w_a[i] V_r(q_a[i]) for the axis a of row r (w: x, y, z
// weights concatenated).  Eight lanes per row: lane l of a row's group takes
// the values i = l, l + 8, ..., then a fixed butterfly sums the eight.
__global__ __launch_bounds__(256) void sep_rows_kernel(const VRowDev* __restrict__ rows, int nrows,
                                                       const double2* __restrict__ w, int3 n, double3 qmin,
                                                       double3 dq, double2* __restrict__ S) {
    const int l8 = threadIdx.x & 7;
    const int r = blockIdx.x * 32 + (threadIdx.x >> 3);
    const bool ok = r < nrows;
    const VRowDev row = rows[ok ? r : 0];
    const int a = row.axis;
    const int na = ok ? (a == 0 ? n.x : (a == 1 ? n.y : n.z)) : 0;
    const int off = a == 0 ? 0 : (a == 1 ? n.x : n.x + n.y);
    const double q0 = a == 0 ? qmin.x : (a == 1 ? qmin.y : qmin.z);
    const double d = a == 0 ? dq.x : (a == 1 ? dq.y : dq.z);
    double sr = 0.0, si = 0.0;
    for (int i = l8; i < na; i += 8) {
        const double2 v = eval_row_fp64(row, q0 + d * (double)i);
        const double2 wi = w[off + i];
        sr += wi.x * v.x - wi.y * v.y;
        si += wi.x * v.y + wi.y * v.x;
    }
    for (int o = 1; o < 8; o <<= 1) {
        sr += __shfl_xor(sr, o);
        si += __shfl_xor(si, o);
    }
    if (ok && l8 == 0) S[r] = make_double2(sr, si);
}

// S[r] = (V(0), V'(0) / i) = (e_0, P e_0 + e_1), both real
__global__ void dip_rows_kernel(const VRowDev* __restrict__ rows, int nrows, double2* __restrict__ S) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += gridDim.x * blockDim.x) {
        const VRowDev row = rows[r];
        S[r] = make_double2(row.e[0], fma(row.P, row.e[0], row.e[1]));
    }
}

// Per packed pair o (unit o / 8, pair o % 8): mode 0 -> G[o] = sum_t Sx Sy Sz
// (complex); mode 1 -> G[4o + c]: c = 0 the value at q = 0 (sum_t a_x a_y a_z),
// c = 1..3 the derivatives / i along x, y, z (a: value, b: derivative / i).
__global__ void sep_pairs_kernel(const int4* __restrict__ slots, const int* __restrict__ coff,
                                 const int* __restrict__ cnpp, int n_units, const double2* __restrict__ S,
                                 int mode, double2* __restrict__ G) {
    const int nv = n_units * kChunk;
    for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < nv; o += gridDim.x * blockDim.x) {
        const int c = o / kChunk, j = o - c * kChunk;
        const int npp = cnpp[c];
        const int4* tc = slots + coff[c] + j * npp;
        if (mode == 0) {
            double2 g = make_double2(0.0, 0.0);
            for (int t = 0; t < npp; ++t) {
                const int4 tr = tc[t];
                if (!tr.w) continue;
                const double2 p = cmul(cmul(S[tr.x], S[tr.y]), S[tr.z]);
                g.x += p.x;
                g.y += p.y;
            }
            G[o] = g;
        } else {
            double v0 = 0.0, dx = 0.0, dy = 0.0, dz = 0.0;
            for (int t = 0; t < npp; ++t) {
                const int4 tr = tc[t];
                if (!tr.w) continue;
                const double2 X = S[tr.x], Y = S[tr.y], Z = S[tr.z];
                v0 += X.x * Y.x * Z.x;
                dx += X.y * Y.x * Z.x;
                dy += X.x * Y.y * Z.x;
                dz += X.x * Y.x * Z.y;
            }
            G[4 * (size_t)o + 0] = make_double2(v0, 0.0);
            G[4 * (size_t)o + 1] = make_double2(dx, 0.0);
            G[4 * (size_t)o + 2] = make_double2(dy, 0.0);
            G[4 * (size_t)o + 3] = make_double2(dz, 0.0);
        }
    }
}

// part[(s * ncomp + c) * nparts + b] = sum over the b-th of nparts slices of
// o of tp64[vcp[o] * ns + s] * G[o * ncomp + c]; one block per (s, c, slice),
// strided partial sums then a fixed tree in LDS.  sep_final_kernel adds the
// slices in order, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void sep_reduce_kernel(const double* __restrict__ tp64, const int* __restrict__ vcp,
                                                         int nv, int ns, const double2* __restrict__ G, int ncomp,
                                                         int nparts, double2* __restrict__ part) {
    __shared__ double2 red[256];
    const int sc = blockIdx.x / nparts, b = blockIdx.x - sc * nparts;
    const int s = sc / ncomp, c = sc - s * ncomp;
    const int per = (nv + nparts - 1) / nparts, o0 = b * per, o1 = min(nv, o0 + per);
    double sr = 0.0, si = 0.0;
    for (int o = o0 + threadIdx.x; o < o1; o += 256) {
        const int k = vcp[o];
        if (k < 0) continue;
        const double t = tp64[(size_t)k * ns + s];
        const double2 g = G[(size_t)o * ncomp + c];
        sr += t * g.x;
        si += t * g.y;
    }
    red[threadIdx.x] = make_double2(sr, si);
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            red[threadIdx.x].x += red[threadIdx.x + h].x;
            red[threadIdx.x].y += red[threadIdx.x + h].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sep_final_kernel(const double2* __restrict__ part, int n, int nparts, double2* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 a = make_double2(0.0, 0.0);
    for (int b = 0; b < nparts; ++b) {
        a.x += part[(size_t)i * nparts + b].x;
        a.y += part[(size_t)i * nparts + b].y;
    }
    out[i] = a;
}

// |f_s(q)|^2 at points, all in FP64: f2[s * nq + i]
__global__ __launch_bounds__(64) void points64_kernel(const VRowDev* __restrict__ rows, const int4* __restrict__ slots,
                                                      const int* __restrict__ coff, const int* __restrict__ cnpp,
                                                      int n_units, const double* __restrict__ tp64,
                                                      const int* __restrict__ vcp, int ns,
                                                      const double* __restrict__ qpts, int nq,
                                                      double* __restrict__ f2) {
    const int iq = blockIdx.x * blockDim.x + threadIdx.x;
    if (iq >= nq) return;
    const double qx = qpts[3 * iq], qy = qpts[3 * iq + 1], qz = qpts[3 * iq + 2];
    double fr[kMaxStates], fi[kMaxStates];
    for (int s = 0; s < kMaxStates; ++s) fr[s] = fi[s] = 0.0;
    for (int c = 0; c < n_units; ++c) {
        const int npp = cnpp[c];
        for (int j = 0; j < kChunk; ++j) {
            const int o = c * kChunk + j;
            const int k = vcp[o];
            if (k < 0) continue;
            const int4* tc = slots + coff[c] + j * npp;
            double2 g = make_double2(0.0, 0.0);
            for (int t = 0; t < npp; ++t) {
                const int4 tr = tc[t];
                if (!tr.w) continue;
                const double2 p =
                    cmul(cmul(eval_row_fp64(rows[tr.x], qx), eval_row_fp64(rows[tr.y], qy)), eval_row_fp64(rows[tr.z], qz));
                g.x += p.x;
                g.y += p.y;
            }
            for (int s = 0; s < ns; ++s) {
                const double t = tp64[(size_t)k * ns + s];
                fr[s] = fma(t, g.x, fr[s]);
                fi[s] = fma(t, g.y, fi[s]);
            }
        }
    }
    for (int s = 0; s < ns; ++s) f2[(size_t)s * nq + iq] = fr[s] * fr[s] + fi[s] * fi[s];
}

int blocks_for(long long n, int b) {
    long long g = (n + b - 1) / b;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

// slices of the transition-weighted reduction per (state, component): about
// 2048 pairs each, at most kSepParts
int sep_parts(int nv) { return std::max(1, std::min(kSepParts, nv / 2048)); }

hipError_t launch_sep_reduce(const double* tp64, const int* vcp, int nv, int ns, const double2* G, int ncomp,
                             double2* part, double2* out, hipStream_t st) {
    const int np = sep_parts(nv);
    hipLaunchKernelGGL(sep_reduce_kernel, dim3(ns * ncomp * np), dim3(256), 0, st, tp64, vcp, nv, ns, G, ncomp, np,
                       part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sep_final_kernel, dim3((ns * ncomp + 63) / 64), dim3(64), 0, st, (const double2*)part,
                       ns * ncomp, np, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_separable(const VRowDev* rows, int nrows, const int4* slots, const int* coff, const int* cnpp,
                            int n_units, const double* tp64, const int* vcp, int ns, const double2* w, const int n[3],
                            const double qmin[3], const double dq[3], double2* S, double2* G, double2* out,
                            hipStream_t st) {
    hipLaunchKernelGGL(sep_rows_kernel, dim3((nrows + 31) / 32), dim3(256), 0, st, rows, nrows, w,
                       make_int3(n[0], n[1], n[2]), make_double3(qmin[0], qmin[1], qmin[2]),
                       make_double3(dq[0], dq[1], dq[2]), S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nv = n_units * kChunk;
    hipLaunchKernelGGL(sep_pairs_kernel, dim3(blocks_for(nv, 256)), dim3(256), 0, st, slots, coff, cnpp, n_units,
                       (const double2*)S, 0, G);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_sep_reduce(tp64, vcp, nv, ns, G, 1, G + nv, out, st);
}

hipError_t launch_dipole(const VRowDev* rows, int nrows, const int4* slots, const int* coff, const int* cnpp,
                         int n_units, const double* tp64, const int* vcp, int ns, double2* S, double2* G,
                         double2* out, hipStream_t st) {
    hipLaunchKernelGGL(dip_rows_kernel, dim3(blocks_for(nrows, 256)), dim3(256), 0, st, rows, nrows, S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nv = n_units * kChunk;
    hipLaunchKernelGGL(sep_pairs_kernel, dim3(blocks_for(nv, 256)), dim3(256), 0, st, slots, coff, cnpp, n_units,
                       (const double2*)S, 1, G);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_sep_reduce(tp64, vcp, nv, ns, G, 4, G + 4 * (size_t)nv, out, st);
}

hipError_t launch_points64(const VRowDev* rows, const int4* slots, const int* coff, const int* cnpp, int n_units,
                           const double* tp64, const int* vcp, int ns, const double* q, int nq, double* f2,
                           hipStream_t st) {
    if (ns < 1 || ns > kMaxStates) return hipErrorInvalidValue;
    hipLaunchKernelGGL(points64_kernel, dim3((nq + 63) / 64), dim3(64), 0, st, rows, slots, coff, cnpp, n_units,
                       tp64, vcp, ns, q, nq, f2);
    return hipGetLastError();
}

}  // namespace scff
