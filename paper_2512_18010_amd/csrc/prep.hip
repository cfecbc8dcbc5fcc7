// Device-side pair precompute and packing (FP64) of the form-factor engine.
//
// Paper Sec. 5.3: the q-independent pair coefficients (eqs. sigmaTidbits,
// positionTidbits, bCoefficients, Mij) are computed once per molecule and
// reused; eq. Ccoefficients gives the monomial form of each 1D polynomial.
// Sec. 5.3 also thresholds Cartesian pair terms per transition; here the
// threshold acts on a q-independent magnitude bound so the dropped part is
// controlled.  Everything below runs on the device from device-resident T:
//
//   rows_kernel     one 1D V-tensor row per (primitive pair, axis, power
//                   pair): P, 1/(4p), e_u (all q-independent factors folded),
//                   and its bound sum_u |e_u| max_q |q|^u e^{-q^2/4p}
//   terms_kernel    per (component pair, primitive pair) term: its 3 rows and
//                   bound; per component pair Tp(s) = (T_mn + T_nm) c_m c_n s_f;
//                   per shell pair the partial sums of |Tp| * bound
//   tot_kernel      tot_s = sum over all terms of |Tp(s)| * bound
//   weight_kernel   w(t) = max_s |Tp(s)| bound(t) / tot_s, integer histogram
//                   of binary exponents
//   thresh_kernel   largest 2^b with sum_{e <= b} count_e 2^e <= eps: dropping
//                   every w < 2^b keeps, for every transition, the dropped
//                   bounds below eps * tot_s
//   count/vkeys     kept terms per component pair, split into virtual pairs
//                   of <= 9 terms, keyed by length (stable radix sort: longest
//                   first, ties in pair order -> deterministic layout)
//   chunk/layout    chunks of 8 virtual pairs, term slots, packed FP32 Tp and
//                   its split-BF16 copy; referenced rows are flagged
//   compact/remap   rows compacted (row 0 = all-zero row for padded slots)
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <cstdint>

#include "engine.h"

namespace scff {

namespace {

__device__ __constant__ int kCartD[3][6][3] = {
    {{0, 0, 0}},
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}},
};

__device__ __forceinline__ int ncart_d(int l) { return (l + 1) * (l + 2) / 2; }

// (u + 2m)! / (m! u! 2^m), u + 2m <= 4
__device__ __forceinline__ double hmono(int u, int m) {
    const double f[5] = {1, 1, 2, 6, 24};
    return f[u + 2 * m] / (f[m] * f[u] * (double)(1 << m));
}

// component pair index within a shell pair -> (c1, c2)
__device__ __forceinline__ void cp_decode(int c, bool same, int ncB, int& c1, int& c2) {
    if (!same) {
        c1 = c / ncB;
        c2 = c - c1 * ncB;
        return;
    }
    // triangular: pairs (c1 <= c2) in row-major order
    int row = 0, rem = c;
    while (rem >= ncB - row) {
        rem -= ncB - row;
        ++row;
    }
    c1 = row;
    c2 = row + rem;
}

constexpr int kHistBias = 1100;   // binary exponents -1100 .. +99
constexpr int kHistBins = 1200;

}  // namespace

// ------------------------------------------------------------------ kernels

__global__ void rows_kernel(const PrepShell* __restrict__ sh, const int4* __restrict__ sp,
                            const double* __restrict__ xyz, const double* __restrict__ exps,
                            const double* __restrict__ coefs, const double* __restrict__ n1d,
                            VRowDev* __restrict__ rows, double* __restrict__ rowsum) {
    const int isp = blockIdx.x;
    const int4 s = sp[isp];   // sA, sB, row_off, term_off
    const PrepShell A_ = sh[s.x], B_ = sh[s.y];
    const int lA = A_.l, lB = B_.l, npb = B_.nprim;
    const int ncls = (lA + 1) * (lB + 1);
    const int nrows = A_.nprim * npb * 3 * ncls;
    const double* A = xyz + 3 * A_.atom;
    const double* B = xyz + 3 * B_.atom;
    const double AB2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
    for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
        const int cls = r % ncls;
        const int ax = (r / ncls) % 3;
        const int pp = r / (3 * ncls);
        const int k = pp / npb, l = pp - k * npb;
        const int i = cls / (lB + 1), j = cls - i * (lB + 1);
        const int ka = A_.off + k, lb = B_.off + l;
        const double al = exps[ka], be = exps[lb];
        const double p = al + be, inv2p = 0.5 / p;
        const double P = (al * A[ax] + be * B[ax]) / p;     // eq. positionTidbits
        const double PA = P - A[ax], PB = P - B[ax];
        const double pa[3] = {1.0, PA, PA * PA}, pb[3] = {1.0, PB, PB * PB};
        const double bin[3][3] = {{1, 0, 0}, {1, 1, 0}, {1, 2, 1}};
        // b_t: coefficients of y^t in (y + PA)^i (y + PB)^j (eq. bCoefficients)
        double bt[5] = {0, 0, 0, 0, 0};
        for (int k1 = 0; k1 <= i; ++k1)
            for (int k2 = 0; k2 <= j; ++k2) bt[k1 + k2] += bin[i][k1] * bin[j][k2] * pa[i - k1] * pb[j - k2];
        // scale: 1D primitive norms; on x also d_k d_l (pi/p)^{3/2} e^{-al be/p |AB|^2} (eq. Mij)
        double scale = n1d[3 * ka + i] * n1d[3 * lb + j];
        if (ax == 0) scale *= coefs[ka] * coefs[lb] * (M_PI / p) * sqrt(M_PI / p) * exp(-al * be / p * AB2);
        VRowDev out{};
        out.P = P;
        out.inv4p = 0.25 / p;
        out.deg = i + j;
        out.axis = ax;
        double sum = 0.0;
        for (int u = 0; u <= i + j; ++u) {
            // e_u of eq. Ccoefficients with sigma_ij^2 = 1/(2p), divided by i^u
            double e = 0.0, pw = 1.0;
            for (int q = 0; q < u; ++q) pw *= inv2p;
            for (int m = 0; u + 2 * m <= i + j; ++m) {
                e += bt[u + 2 * m] * hmono(u, m) * pw;
                pw *= inv2p;
            }
            out.e[u] = e * scale;
            // max_q |q|^u exp(-q^2/(4p)) = (2 p u / e)^{u/2}
            const double mpk = u == 0 ? 1.0 : pow(2.0 * p * u / M_E, 0.5 * u);
            sum += fabs(out.e[u]) * mpk;
        }
        rows[s.z + r] = out;
        rowsum[s.z + r] = sum;
    }
}

__global__ void terms_kernel(const PrepShell* __restrict__ sh, const int4* __restrict__ sp,
                             const int* __restrict__ sp_cp, const int* __restrict__ bf0,
                             const double* __restrict__ cnorm, const double* __restrict__ rowsum,
                             const double* __restrict__ T, int nbf, int ns, double spin,
                             int4* __restrict__ trow, double* __restrict__ tbound,
                             int2* __restrict__ cpmn, double* __restrict__ tp64,
                             double* __restrict__ bsum, double* __restrict__ part) {
    const int isp = blockIdx.x;
    const int4 s = sp[isp];
    const PrepShell A_ = sh[s.x], B_ = sh[s.y];
    const int lA = A_.l, lB = B_.l;
    const int npp = A_.nprim * B_.nprim;
    const int ncls = (lA + 1) * (lB + 1);
    const bool same = s.x == s.y;
    const int ncA = ncart_d(lA), ncB = ncart_d(lB);
    const int ncp = same ? ncA * (ncA + 1) / 2 : ncA * ncB;
    const int cp0 = sp_cp[isp];
    // terms and their bounds
    for (int t = threadIdx.x; t < ncp * npp; t += blockDim.x) {
        const int c = t / npp, pp = t - c * npp;
        int c1, c2;
        cp_decode(c, same, ncB, c1, c2);
        const int* pA = kCartD[lA][c1];
        const int* pB = kCartD[lB][c2];
        int rr[3];
        double bd = 1.0;
        for (int ax = 0; ax < 3; ++ax) {
            rr[ax] = s.z + pp * 3 * ncls + ax * ncls + pA[ax] * (lB + 1) + pB[ax];
            bd *= rowsum[rr[ax]];
        }
        trow[s.w + t] = make_int4(rr[0], rr[1], rr[2], cp0 + c);
        tbound[s.w + t] = bd;
    }
    __syncthreads();
    // component pairs: mu, nu, packed weights and the sum of their term bounds
    for (int c = threadIdx.x; c < ncp; c += blockDim.x) {
        int c1, c2;
        cp_decode(c, same, ncB, c1, c2);
        const int mu = bf0[s.x] + c1, nu = bf0[s.y] + c2;
        cpmn[cp0 + c] = make_int2(mu, nu);
        double b = 0.0;
        for (int pp = 0; pp < npp; ++pp) b += tbound[s.w + c * npp + pp];
        bsum[cp0 + c] = b;
        const double cc = cnorm[mu] * cnorm[nu] * spin;
        for (int st = 0; st < ns; ++st) {
            const double* Ts = T + (size_t)st * nbf * nbf;
            const double v = mu == nu ? Ts[(size_t)mu * nbf + mu] : Ts[(size_t)mu * nbf + nu] + Ts[(size_t)nu * nbf + mu];
            tp64[(size_t)(cp0 + c) * ns + st] = v * cc;
        }
    }
    __syncthreads();
    // per shell pair partial of sum_t |Tp(s)| bound(t), fixed order
    for (int st = threadIdx.x; st < ns; st += blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c < ncp; ++c) acc += fabs(tp64[(size_t)(cp0 + c) * ns + st]) * bsum[cp0 + c];
        part[(size_t)isp * ns + st] = acc;
    }
}

__global__ void tot_kernel(const double* __restrict__ part, int nsp, int ns, double* __restrict__ tot) {
    // one block of 256 threads per state: fixed-order strided partial sums,
    // then a fixed-shape tree (deterministic)
    __shared__ double red[256];
    for (int st = blockIdx.x; st < ns; st += gridDim.x) {
        double a = 0.0;
        for (int i = threadIdx.x; i < nsp; i += blockDim.x) a += part[(size_t)i * ns + st];
        red[threadIdx.x] = a;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) tot[st] = red[0];
        __syncthreads();
    }
}

// per component pair: m_k = max_s |Tp(s,k)| / tot_s
__global__ void pairmax_kernel(const double* __restrict__ tp64, const double* __restrict__ tot, int ns, int ncp,
                               double* __restrict__ mk) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ncp; k += gridDim.x * blockDim.x) {
        double m = 0.0;
        for (int st = 0; st < ns; ++st)
            if (tot[st] > 0.0) m = fmax(m, fabs(tp64[(size_t)k * ns + st]) / tot[st]);
        mk[k] = m;
    }
}

__global__ void weight_kernel(const int4* __restrict__ trow, const double* __restrict__ tbound,
                              const double* __restrict__ mk, long long nterms, double* __restrict__ w,
                              unsigned int* __restrict__ hist) {
    // the workgroup counts its terms' exponents in LDS (most terms share a
    // few bins, so global atomics per term would serialise) and adds its
    // non-empty bins to the global histogram once
    __shared__ unsigned int lh[kHistBins];
    for (int b = threadIdx.x; b < kHistBins; b += blockDim.x) lh[b] = 0u;
    __syncthreads();
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < nterms;
         t += (long long)gridDim.x * blockDim.x) {
        const double x = mk[trow[t].w] * tbound[t];
        w[t] = x;
        if (x > 0.0) {
            int e;
            frexp(x, &e);    // x in [2^(e-1), 2^e)
            e = min(max(e + kHistBias, 0), kHistBins - 1);
            atomicAdd(&lh[e], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kHistBins; b += blockDim.x)
        if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

__global__ void thresh_kernel(const unsigned int* __restrict__ hist, double eps, double* __restrict__ thr) {
    // one wave: per-bin upper bounds in LDS, then the largest bin `best` such
    // that the bounds of all bins <= best sum to at most eps.  The bins are
    // scanned in order as 64 runs of consecutive bins (one run per lane):
    // each lane sums its run, lane 0 adds the run sums in order until the
    // total would pass eps and then walks that run bin by bin (83 serial
    // steps instead of 1200; a fixed order, so the result is deterministic)
    constexpr int kRun = (kHistBins + 63) / 64;
    __shared__ double pre[kHistBins];
    __shared__ double run[64];
    const int lane = threadIdx.x;
    for (int b = lane; b < kHistBins; b += blockDim.x) pre[b] = (double)hist[b] * ldexp(1.0, b - kHistBias);
    __syncthreads();
    if (lane < 64) {
        double sr = 0.0;
        for (int b = lane * kRun; b < min((lane + 1) * kRun, kHistBins); ++b) sr += pre[b];
        run[lane] = sr;
    }
    __syncthreads();
    if (lane == 0) {
        if (!(eps > 0.0)) {
            thr[0] = -1.0;   // no screening: keep every term, zero or not
            return;
        }
        double sum = 0.0;
        int r = 0;
        while (r < 64 && sum + run[r] <= eps) sum += run[r++];
        int best = r * kRun - 1;   // every bin of the runs before r is dropped
        if (r < 64) {
            for (int b = r * kRun; b < min((r + 1) * kRun, kHistBins); ++b) {
                if (sum + pre[b] > eps) break;
                sum += pre[b];
                best = b;
            }
        }
        best = min(best, kHistBins - 1);
        // w < 2^(best - bias) exactly when its frexp exponent bin is <= best
        thr[0] = best < 0 ? 0.0 : ldexp(1.0, best - kHistBias);
    }
}

__device__ __forceinline__ bool term_kept(double w, double thr) {
    return thr < 0.0 || (w > 0.0 && w >= thr);
}

__global__ void count_kernel(const int* __restrict__ cp_first, const int* __restrict__ cp_nterms,
                             const double* __restrict__ w, const double* __restrict__ thr, int ncp,
                             int* __restrict__ nk, int* __restrict__ nv,
                             unsigned long long* __restrict__ stats) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ncp; k += gridDim.x * blockDim.x) {
        const double th = thr[0];
        int n = 0;
        for (int t = 0; t < cp_nterms[k]; ++t) n += term_kept(w[cp_first[k] + t], th) ? 1 : 0;
        nk[k] = n;
        nv[k] = (n + kMaxTermsPerPair - 1) / kMaxTermsPerPair;
        if (n > 0) {
            atomicAdd(&stats[0], 1ull);                 // K
            atomicAdd(&stats[1], (unsigned long long)n); // R
        }
    }
}

__global__ void vkeys_kernel(const int* __restrict__ nk, const int* __restrict__ nv,
                             const int* __restrict__ vbase, int ncp, unsigned int* __restrict__ key,
                             int* __restrict__ val, int4* __restrict__ vinfo) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ncp; k += gridDim.x * blockDim.x) {
        const int n = nk[k], m = nv[k];
        int pos = 0;
        for (int v = 0; v < m; ++v) {
            const int take = (n - pos) / (m - v);
            const int id = vbase[k] + v;
            key[id] = (unsigned)(kMaxTermsPerPair - take);   // longest first
            val[id] = id;
            vinfo[id] = make_int4(k, pos, take, 0);
            pos += take;
        }
    }
}

__global__ void unit_kernel(const int* __restrict__ order, const int4* __restrict__ vinfo, int nv,
                            int n_chunks, int* __restrict__ cnpp, int* __restrict__ csize,
                            int* __restrict__ uhist) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n_chunks; c += gridDim.x * blockDim.x) {
        const int o = c * kChunk;
        const int npp = o < nv ? max(1, vinfo[order[o]].z) : 1;
        cnpp[c] = npp;
        csize[c] = kChunk * npp;
        atomicAdd(&uhist[npp], 1);   // units per term count (units are sorted by it, longest first)
    }
}

__global__ void layout_kernel(const int* __restrict__ order, const int4* __restrict__ vinfo, int nv,
                              int n_vpairs, const int* __restrict__ cnpp, const int* __restrict__ coff,
                              const int* __restrict__ cp_first, const int* __restrict__ cp_nterms,
                              const int4* __restrict__ trow, const double* __restrict__ w,
                              const double* __restrict__ thr, const double* __restrict__ tp64, int ns,
                              int SW, int4* __restrict__ slots, float* __restrict__ tp32,
                              uint32_t* __restrict__ tpbf, int* __restrict__ row_used, int* __restrict__ vcp) {
    for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < n_vpairs; o += gridDim.x * blockDim.x) {
        const int c = o / kChunk, j = o - c * kChunk;
        const int npp = cnpp[c];
        int4* dst = slots + coff[c] + j * npp;
        int len = 0, k = -1;
        if (o < nv) {
            const int4 vi = vinfo[order[o]];
            k = vi.x;
            len = vi.z;
            const double th = thr[0];
            int seen = 0, q = 0;
            for (int t = 0; t < cp_nterms[k] && q < len; ++t) {
                const int ti = cp_first[k] + t;
                if (!term_kept(w[ti], th)) continue;
                if (seen++ < vi.y) continue;
                const int4 tr = trow[ti];
                dst[q++] = make_int4(tr.x, tr.y, tr.z, 1);
                row_used[tr.x] = 1;
                row_used[tr.y] = 1;
                row_used[tr.z] = 1;
            }
        }
        for (int q = len; q < npp; ++q) dst[q] = make_int4(-1, -1, -1, 0);
        vcp[o] = k;   // component pair of this packed pair (-1: padding), for the FP64 weights
        for (int st = 0; st < SW; ++st) {
            const float v = (k >= 0 && st < ns) ? (float)tp64[(size_t)k * ns + st] : 0.0f;
            tp32[(size_t)o * SW + st] = v;
            // split-BF16: hi = RNE(v), lo = RNE(v - hi); packed (hi | lo << 16)
            const uint32_t u = __float_as_uint(v);
            const uint32_t hi = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
            const float r = v - __uint_as_float(hi << 16);
            const uint32_t ur = __float_as_uint(r);
            const uint32_t lo = (ur + 0x7fffu + ((ur >> 16) & 1u)) >> 16;
            tpbf[(size_t)o * SW + st] = hi | (lo << 16);
        }
    }
}

__global__ void compact_kernel(const VRowDev* __restrict__ rows, const int* __restrict__ used,
                               const int* __restrict__ newid, int nrows, VRowDev* __restrict__ out) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += gridDim.x * blockDim.x) {
        if (r == 0) {
            VRowDev z{};
            z.inv4p = 1.0;
            out[0] = z;
        }
        if (used[r]) out[1 + newid[r]] = rows[r];
    }
}

__global__ void remap_kernel(int4* __restrict__ slots, long long nslots, const int* __restrict__ newid) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nslots;
         i += (long long)gridDim.x * blockDim.x) {
        int4 s = slots[i];
        if (s.w) s = make_int4(1 + newid[s.x], 1 + newid[s.y], 1 + newid[s.z], 1);
        else s = make_int4(0, 0, 0, 0);
        slots[i] = s;
    }
}

// ------------------------------------------------------------------ host driver

namespace {

int blocks_for(long long n, int bs) {
    long long b = (n + bs - 1) / bs;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (int)b;
}

}  // namespace

// Runs the whole precompute on `st`.  Buffers in `w` are (re)allocated through
// `alloc`, which enforces the caller's memory budget.  Returns hipSuccess or
// the first HIP error; sizes and statistics are written to `res`.
hipError_t run_prep(const PrepInputs& in, PrepWork& w, PrepResult& res, hipStream_t st,
                    const std::function<hipError_t(DeviceBuffer&, size_t)>& alloc) {
    hipError_t e;
#define CK(x)                                  \
    do {                                       \
        if ((e = (x)) != hipSuccess) return e; \
    } while (0)
    const long long NR = in.n_rows_all, NT = in.n_terms_all;
    const int NCP = in.n_cp, NSP = in.n_sp, ns = in.n_states;
    const int SW = kStateBlock * ((ns + kStateBlock - 1) / kStateBlock);
    CK(alloc(w.rows_all, (size_t)NR * sizeof(VRowDev)));
    CK(alloc(w.rowsum, (size_t)NR * sizeof(double)));
    CK(alloc(w.trow, (size_t)NT * sizeof(int4)));
    CK(alloc(w.tbound, (size_t)NT * sizeof(double)));
    CK(alloc(w.wt, (size_t)NT * sizeof(double)));
    CK(alloc(w.cpmn, (size_t)NCP * sizeof(int2)));
    CK(alloc(w.tp64, (size_t)NCP * ns * sizeof(double)));
    CK(alloc(w.bsum, (size_t)NCP * sizeof(double)));
    CK(alloc(w.part, (size_t)NSP * ns * sizeof(double)));
    CK(alloc(w.small, 4096 + kHistBins * sizeof(unsigned) + 64));
    CK(alloc(w.nk, (size_t)NCP * sizeof(int)));
    CK(alloc(w.nv, (size_t)NCP * sizeof(int)));
    CK(alloc(w.vbase, (size_t)NCP * sizeof(int)));
    double* tot = (double*)w.small.p;                                    // [<= 32]
    double* thr = tot + 64;                                              // [1]
    unsigned long long* stats = (unsigned long long*)(thr + 8);          // [2]
    unsigned* hist = (unsigned*)((char*)w.small.p + 4096);               // [kHistBins]

    CK(hipMemsetAsync(w.small.p, 0, w.small.bytes, st));
    hipLaunchKernelGGL(rows_kernel, dim3(NSP), dim3(128), 0, st, in.shells, in.sp, in.xyz, in.exps,
                       in.coefs, in.n1d, (VRowDev*)w.rows_all.p, (double*)w.rowsum.p);
    CK(hipGetLastError());
    hipLaunchKernelGGL(terms_kernel, dim3(NSP), dim3(128), 0, st, in.shells, in.sp, in.sp_cp, in.bf0,
                       in.cnorm, (const double*)w.rowsum.p, in.T, in.nbf, ns, in.spin,
                       (int4*)w.trow.p, (double*)w.tbound.p, (int2*)w.cpmn.p, (double*)w.tp64.p,
                       (double*)w.bsum.p, (double*)w.part.p);
    CK(hipGetLastError());
    hipLaunchKernelGGL(tot_kernel, dim3(ns), dim3(256), 0, st, (const double*)w.part.p, NSP, ns, tot);
    CK(hipGetLastError());
    hipLaunchKernelGGL(pairmax_kernel, dim3(blocks_for(NCP, 256)), dim3(256), 0, st, (const double*)w.tp64.p,
                       (const double*)tot, ns, NCP, (double*)w.bsum.p);
    CK(hipGetLastError());
    hipLaunchKernelGGL(weight_kernel, dim3(std::min(blocks_for(NT, 256), 512)), dim3(256), 0, st, (const int4*)w.trow.p,
                       (const double*)w.tbound.p, (const double*)w.bsum.p, NT, (double*)w.wt.p, hist);
    CK(hipGetLastError());
    hipLaunchKernelGGL(thresh_kernel, dim3(1), dim3(64), 0, st, (const unsigned*)hist, in.eps, thr);
    CK(hipGetLastError());
    hipLaunchKernelGGL(count_kernel, dim3(blocks_for(NCP, 256)), dim3(256), 0, st, in.cp_first,
                       in.cp_nterms, (const double*)w.wt.p, (const double*)thr, NCP, (int*)w.nk.p,
                       (int*)w.nv.p, stats);
    CK(hipGetLastError());
    // exclusive scan of virtual pairs per component pair
    size_t tmp_bytes = 0;
    CK(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, (int*)w.nv.p, (int*)w.vbase.p, NCP, st));
    CK(alloc(w.tmp, tmp_bytes + 256));
    CK(hipcub::DeviceScan::ExclusiveSum(w.tmp.p, tmp_bytes, (int*)w.nv.p, (int*)w.vbase.p, NCP, st));
    // readbacks of sizes land in the context's pinned host memory when it has
    // some (a DMA; pageable destinations are staged by the runtime)
    alignas(16) unsigned char local_rb[256];
    unsigned char* rb = w.pinned ? (unsigned char*)w.pinned : local_rb;
    int* last = (int*)rb;                                  // [2]
    unsigned long long* kr = (unsigned long long*)(rb + 16);   // [2]
    int* lastc = (int*)(rb + 32);                          // [2]
    int* uhist = (int*)(rb + 64);                          // [16]
    int* lastr = (int*)(rb + 128);                         // [2]
    // total virtual pairs, K and R
    CK(hipMemcpyAsync(&last[0], (int*)w.vbase.p + NCP - 1, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&last[1], (int*)w.nv.p + NCP - 1, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(kr, stats, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    const int NV = last[0] + last[1];
    res.pairs_kept = (long long)kr[0];
    res.terms_kept = (long long)kr[1];
    const int NVA = NV > 0 ? NV : 1;
    CK(alloc(w.key, (size_t)NVA * sizeof(unsigned) * 2));
    CK(alloc(w.val, (size_t)NVA * sizeof(int) * 2));
    CK(alloc(w.vinfo, (size_t)NVA * sizeof(int4)));
    unsigned* key_in = (unsigned*)w.key.p;
    unsigned* key_out = key_in + NVA;
    int* val_in = (int*)w.val.p;
    int* val_out = val_in + NVA;
    if (NV > 0) {
        hipLaunchKernelGGL(vkeys_kernel, dim3(blocks_for(NCP, 256)), dim3(256), 0, st, (const int*)w.nk.p,
                           (const int*)w.nv.p, (const int*)w.vbase.p, NCP, key_in, val_in, (int4*)w.vinfo.p);
        CK(hipGetLastError());
        size_t sort_bytes = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, key_in, key_out, val_in, val_out, NV, 0, 4, st));
        CK(alloc(w.tmp2, sort_bytes + 256));
        CK(hipcub::DeviceRadixSort::SortPairs(w.tmp2.p, sort_bytes, key_in, key_out, val_in, val_out, NV, 0, 4, st));
    }
    // units of kChunk sorted virtual pairs, each padded to its first pair's term count
    const int n_vpairs = ((NVA + kChunk - 1) / kChunk) * kChunk;
    const int n_chunks = n_vpairs / kChunk;   // units
    CK(alloc(w.cnpp, (size_t)n_chunks * sizeof(int)));
    CK(alloc(w.csize, (size_t)n_chunks * sizeof(int)));
    CK(alloc(w.coff, (size_t)n_chunks * sizeof(int)));
    CK(alloc(w.uhist, 16 * sizeof(int)));
    CK(hipMemsetAsync(w.uhist.p, 0, 16 * sizeof(int), st));
    hipLaunchKernelGGL(unit_kernel, dim3(blocks_for(n_chunks, 256)), dim3(256), 0, st, (const int*)val_out,
                       (const int4*)w.vinfo.p, NV, n_chunks, (int*)w.cnpp.p, (int*)w.csize.p, (int*)w.uhist.p);
    CK(hipGetLastError());
    size_t tmp3 = 0;
    CK(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp3, (int*)w.csize.p, (int*)w.coff.p, n_chunks, st));
    CK(alloc(w.tmp3, tmp3 + 256));
    CK(hipcub::DeviceScan::ExclusiveSum(w.tmp3.p, tmp3, (int*)w.csize.p, (int*)w.coff.p, n_chunks, st));
    CK(hipMemcpyAsync(&lastc[0], (int*)w.coff.p + n_chunks - 1, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&lastc[1], (int*)w.csize.p + n_chunks - 1, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(uhist, w.uhist.p, 16 * sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    // grid-kernel chunks: runs of consecutive units with equal npp (units come
    // longest first), at most kMaxUnitsPerChunk units and kMaxChunkTerms terms.
    // Entry = (first unit, units, npp, first term slot); the slot offsets of
    // the units follow from the same counts (kChunk * npp slots per unit).
    std::vector<int>& ch = w.chunk_host;
    ch.clear();
    {
        int u0 = 0;
        long long slot = 0;
        for (int v = kMaxTermsPerPair; v >= 1; --v) {
            const int cnt = uhist[v];
            int um = kMaxChunkTerms / (kChunk * v);
            if (um > kMaxUnitsPerChunk) um = kMaxUnitsPerChunk;
            for (int k = 0; k < cnt; k += um) {
                const int nu = cnt - k < um ? cnt - k : um;
                ch.push_back(u0 + k);
                ch.push_back(nu);
                ch.push_back(v);
                ch.push_back((int)slot);
                slot += (long long)nu * kChunk * v;
            }
            u0 += cnt;
        }
        // every unit has 1 <= npp <= kMaxTermsPerPair; slots agree with the device scan
        if (u0 != n_chunks || slot != (long long)lastc[0] + lastc[1]) return hipErrorUnknown;
    }
    const int n_grid_chunks = (int)(ch.size() / 4);
    CK(alloc(w.chunks, ch.size() * sizeof(int)));
    {
        // through pinned memory when it fits; the copy is complete at the
        // synchronisation below, before the buffer can be written again
        const size_t cb = ch.size() * sizeof(int);
        const void* src = ch.data();
        if (w.pinned && cb <= kPinnedBytes - kPinnedTables) {
            std::memcpy((unsigned char*)w.pinned + kPinnedTables, ch.data(), cb);
            src = (unsigned char*)w.pinned + kPinnedTables;
        }
        CK(hipMemcpyAsync(w.chunks.p, src, cb, hipMemcpyHostToDevice, st));
    }
    const long long nslots = (long long)lastc[0] + lastc[1];
    CK(alloc(w.slots, (size_t)nslots * sizeof(int4)));
    CK(alloc(w.tp32, (size_t)n_vpairs * SW * sizeof(float)));
    CK(alloc(w.tpbf, (size_t)n_vpairs * SW * sizeof(uint32_t)));
    CK(alloc(w.vcp, (size_t)n_vpairs * sizeof(int)));
    CK(alloc(w.row_used, (size_t)NR * sizeof(int)));
    CK(alloc(w.newid, (size_t)NR * sizeof(int)));
    CK(hipMemsetAsync(w.row_used.p, 0, (size_t)NR * sizeof(int), st));
    hipLaunchKernelGGL(layout_kernel, dim3(blocks_for(n_vpairs, 128)), dim3(128), 0, st, (const int*)val_out,
                       (const int4*)w.vinfo.p, NV, n_vpairs, (const int*)w.cnpp.p, (const int*)w.coff.p,
                       in.cp_first, in.cp_nterms, (const int4*)w.trow.p, (const double*)w.wt.p,
                       (const double*)thr, (const double*)w.tp64.p, ns, SW, (int4*)w.slots.p,
                       (float*)w.tp32.p, (uint32_t*)w.tpbf.p, (int*)w.row_used.p, (int*)w.vcp.p);
    CK(hipGetLastError());
    size_t tmp4 = 0;
    CK(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp4, (int*)w.row_used.p, (int*)w.newid.p, (int)NR, st));
    CK(alloc(w.tmp4, tmp4 + 256));
    CK(hipcub::DeviceScan::ExclusiveSum(w.tmp4.p, tmp4, (int*)w.row_used.p, (int*)w.newid.p, (int)NR, st));
    CK(hipMemcpyAsync(&lastr[0], (int*)w.newid.p + NR - 1, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&lastr[1], (int*)w.row_used.p + NR - 1, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    const int nrows_used = lastr[0] + lastr[1];
    CK(alloc(w.rows, (size_t)(nrows_used + 1) * sizeof(VRowDev)));
    hipLaunchKernelGGL(compact_kernel, dim3(blocks_for(NR, 256)), dim3(256), 0, st, (const VRowDev*)w.rows_all.p,
                       (const int*)w.row_used.p, (const int*)w.newid.p, (int)NR, (VRowDev*)w.rows.p);
    CK(hipGetLastError());
    hipLaunchKernelGGL(remap_kernel, dim3(blocks_for(nslots, 256)), dim3(256), 0, st, (int4*)w.slots.p, nslots,
                       (const int*)w.newid.p);
    CK(hipGetLastError());
    res.n_vpairs = n_vpairs;
    res.n_units = n_chunks;
    res.n_chunks = n_grid_chunks;
    res.n_slots = nslots;
    res.n_rows = nrows_used + 1;
    res.state_blocks = SW / kStateBlock;
    return hipSuccess;
#undef CK
}

}  // namespace scff
