// The spherical method (paper Sec. 4 eqs. DTensor, WTensor, YYY,
// SphericalMethod, RTensor; Sec. 5.4; App. B) on the device, FP64:
//
//   sph_geom_kernel    per geometry g (a primitive pair of a shell pair, so
//                      one Gaussian centre P_g and exponent p_g): the
//                      W tensor summed over the geometry's component pairs
//                      with their packed transition weights,
//                        W^s_g[n lam mu] = sum_c Tp_s(c) sum_{u+v+w=n} D_c^{uvw} Theta^{uvw}_{lam mu},
//                      D_c^{uvw} = i^n e^x_u e^y_v e^z_w from the 1D rows of the
//                      pair precompute; and 4 pi i^L Y_L^M*(P^_g) for L <= lmax + 4;
//   sph_q_kernel       for each radius q, the contraction over geometries
//                        Q^s[lam mu][L M](q) = sum_g b^s_g[lam mu](q) a_g[L M](q),
//                        b = e^{-q^2/4p} sum_n q^n W^s_g[n lam mu],
//                        a = 4 pi i^L j_L(q |P_g|) Y_L^M*(P^_g),
//                      a complex GEMM on the FP64 matrix cores (rows: state x
//                      (lam mu), columns: (L M), k: geometries) tiled in LDS, with the spherical
//                      Bessel functions j_L(q |P_g|) (sph_bessel_kernel: Miller's
//                      downward recurrence from far above max(L, x), normalised
//                      with j_0 = sin x / x or j_1, whichever is larger; the
//                      two-term power series below x = 1e-4);
//   sph_couple_kernel  R^s_lm(q) = sum_{lam mu, L} G^{mu, m-mu}_{lam L l} Q^s[lam mu][L, m-mu]
//                      (eq. RTensor with the Gaunt coefficients of eq. YYY);
//   sph_legendre_kernel / sph_phi_kernel
//                      the angular grid f^s(q, theta_i, phi_j) = sum_lm R_lm Y_l^m
//                      (eq. SphericalMethod) as a Legendre stage per theta and a
//                      Fourier stage per phi; sph_avg_kernel <|f|^2>_Omega.
#include <hip/hip_runtime.h>

#include "engine.h"

namespace scff {

namespace {

constexpr int kLam = (kSphMaxN + 1) * (kSphMaxN + 1);   // 25 harmonics lam <= 4

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// i^n
__device__ __forceinline__ double2 ipow(int n) {
    switch (n & 3) {
        case 0: return make_double2(1.0, 0.0);
        case 1: return make_double2(0.0, 1.0);
        case 2: return make_double2(-1.0, 0.0);
        default: return make_double2(0.0, -1.0);
    }
}

// 4 pi i^L Y_L^M*(theta, phi) for L <= Lmax into out[L^2 + L + M] (the
// plane-wave factor of the contraction with the harmonic; Condon-Shortley,
// orthonormal; associated Legendre functions by upward recurrence in L).
__device__ void ylm_conj_row(int Lmax, double theta, double phi, double2* out) {
    double sn, cs;
    sincos(theta, &sn, &cs);
    double pmm = sqrt(1.0 / (4.0 * M_PI));
    for (int m = 0; m <= Lmax; ++m) {
        if (m > 0) pmm *= -sqrt((2.0 * m + 1.0) / (2.0 * m)) * sn;
        double es, ec;
        sincos(m * phi, &es, &ec);
        double p2 = 0.0, p1 = pmm;
        for (int l = m; l <= Lmax; ++l) {
            double cur;
            if (l == m) {
                cur = pmm;
            } else if (l == m + 1) {
                cur = sqrt(2.0 * m + 3.0) * cs * pmm;
            } else {
                const double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
                const double b = sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
                cur = a * (cs * p1 - b * p2);
            }
            if (l > m) {
                p2 = p1;
                p1 = cur;
            }
            // conj(Y_l^m) = cur e^{-i m phi};  conj(Y_l^{-m}) = (-1)^m cur e^{+i m phi}
            const double2 f = cscale(ipow(l), 4.0 * M_PI);
            out[l * l + l + m] = cmul(f, make_double2(cur * ec, -cur * es));
            if (m > 0) {
                const double sg = (m & 1) ? -1.0 : 1.0;
                out[l * l + l - m] = cmul(f, make_double2(sg * cur * ec, sg * cur * es));
            }
        }
    }
}

__global__ __launch_bounds__(128) void sph_geom_kernel(const SphGeom* __restrict__ geo, int n_geo,
                                                       const VRowDev* __restrict__ rows,
                                                       const int4* __restrict__ trow,
                                                       const double* __restrict__ tp64, int ns,
                                                       const double2* __restrict__ theta, const int* __restrict__ uvw_idx,
                                                       const int* __restrict__ nfirst, int n_nlm, int Lmax,
                                                       double4* __restrict__ gdat, double2* __restrict__ Yc,
                                                       double2* __restrict__ W) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_geo) return;
    const SphGeom G = geo[g];
    // W[(b ns + s) n_geo + g]: geometries fastest, so the contraction kernel's
    // loads of one (b, s) over a chunk of geometries are contiguous
    double2* Wg = W + g;
    for (int i = 0; i < n_nlm * ns; ++i) Wg[(size_t)i * n_geo] = make_double2(0.0, 0.0);
    const int4 t0 = trow[G.term0 + G.pp];
    const double Px = rows[t0.x].P, Py = rows[t0.y].P, Pz = rows[t0.z].P;
    const double d = sqrt(Px * Px + Py * Py + Pz * Pz);
    const double th = d > 0.0 ? acos(fmin(1.0, fmax(-1.0, Pz / d))) : 0.0;
    const double ph = d > 0.0 ? atan2(Py, Px) : 0.0;
    gdat[g] = make_double4(d, th, ph, rows[t0.x].inv4p);
    ylm_conj_row(Lmax, th, ph, Yc + (size_t)g * (Lmax + 1) * (Lmax + 1));
    for (int c = 0; c < G.ncp; ++c) {
        const int4 tr = trow[G.term0 + c * G.npp + G.pp];
        const VRowDev& rx = rows[tr.x];
        const VRowDev& ry = rows[tr.y];
        const VRowDev& rz = rows[tr.z];
        const double* tp = tp64 + (size_t)tr.w * ns;
        for (int u = 0; u <= rx.deg; ++u)
            for (int v = 0; v <= ry.deg; ++v)
                for (int w = 0; w <= rz.deg; ++w) {
                    const double e = rx.e[u] * ry.e[v] * rz.e[w];
                    if (e == 0.0) continue;
                    const int n = u + v + w;
                    const int a = uvw_idx[(u * (kSphMaxN + 1) + v) * (kSphMaxN + 1) + w];
                    const double2 coef = cscale(ipow(n), e);
                    for (int b = nfirst[n]; b < nfirst[n + 1]; ++b) {
                        const double2 th_ab = theta[(size_t)a * n_nlm + b];
                        if (th_ab.x == 0.0 && th_ab.y == 0.0) continue;
                        const double2 x = cmul(coef, th_ab);
                        for (int s = 0; s < ns; ++s) {
                            double2& o = Wg[((size_t)b * ns + s) * n_geo];
                            o.x += tp[s] * x.x;
                            o.y += tp[s] * x.y;
                        }
                    }
                }
    }
}

// Spherical Bessel functions and Gaussian of every (radius, geometry):
// J[(iq (Lmax + 2) + L) n_geo + g] = j_L(q |P_g|) for L <= Lmax and, at
// L = Lmax + 1, e^{-q^2 / 4p_g}.  One thread per (radius, geometry); the
// recurrence of bessel_range, written straight to the strided table.
__global__ void sph_bessel_kernel(const double4* __restrict__ gdat, int n_geo, int Lmax, const double* __restrict__ qs,
                                  int n_q, double* __restrict__ J) {
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)n_q * n_geo) return;
    const int g = (int)(idx % n_geo), iq = (int)(idx / n_geo);
    const double4 gg = gdat[g];
    const double q = qs[iq], x = q * gg.x;
    double* o = J + (size_t)iq * (Lmax + 2) * n_geo + g;
    o[(size_t)(Lmax + 1) * n_geo] = exp(-q * q * gg.w);
    if (x < 1e-4) {
        double df = 1.0, xl = 1.0;
        for (int L = 0; L <= Lmax; ++L) {
            if (L > 0) {
                df *= 2.0 * L + 1.0;
                xl *= x;
            }
            o[(size_t)L * n_geo] = xl / df * (1.0 - x * x / (2.0 * (2.0 * L + 3.0)));
        }
        return;
    }
    const int N = max(Lmax, (int)x) + 32;
    const double rx = 1.0 / x;
    double fp = 0.0, f = 1e-280, f1 = 0.0;
    for (int L = N; L >= 1; --L) {
        const double fm = (2.0 * L + 1.0) * rx * f - fp;   // f_{L-1}
        fp = f;
        f = fm;
        if (L - 1 <= Lmax) o[(size_t)(L - 1) * n_geo] = f;
        if (L - 1 == 1) f1 = f;
        if (fabs(f) > 1e250) {   // rescale everything kept so far
            f *= 1e-250;
            fp *= 1e-250;
            f1 *= 1e-250;
            for (int k = L - 1; k <= Lmax; ++k) o[(size_t)k * n_geo] *= 1e-250;
        }
    }
    double sn, cs;
    sincos(x, &sn, &cs);
    const double j0 = sn * rx, j1 = (sn * rx - cs) * rx;
    const double scale = fabs(j0) >= fabs(j1) ? j0 / f : j1 / f1;
    for (int L = 0; L <= Lmax; ++L) o[(size_t)L * n_geo] *= scale;
}

// Row operands of the contraction for a batch of nqb radii from iq0 on,
//   Bq[(k nrows + row) n_geo + g] = e^{-q^2/4p_g} sum_n q^n W^s_g[n lam mu],
// row = (s, lam mu), q = qs[iq0 + k]; the Gaussian is row Lmax + 1 of the
// radius's Bessel table.  One thread per (row, geometry): its W values (n =
// lam, lam + 2, .. <= 4) are loaded once for the batch.
__global__ __launch_bounds__(256) void sph_b_kernel(const double2* __restrict__ W, const double* __restrict__ J,
                                                    const int* __restrict__ nlm_of, int n_geo, int ns, int Lmax,
                                                    const double* __restrict__ qs, int iq0, int nqb,
                                                    double2* __restrict__ Bq) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_geo) return;
    const int row = blockIdx.y, nrows = ns * kLam;
    const int st = row / kLam, lm = row - st * kLam;
    const int lam = lm < 1 ? 0 : lm < 4 ? 1 : lm < 9 ? 2 : lm < 16 ? 3 : 4;
    // slots m = 0..2 hold n = lam + 2 m (those above kSphMaxN are zero)
    double2 w[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int n = lam + 2 * m;
        w[m] = n <= kSphMaxN ? W[((size_t)nlm_of[n * kLam + lm] * ns + st) * n_geo + g] : make_double2(0.0, 0.0);
    }
    for (int k = 0; k < nqb; ++k) {
        const int iq = iq0 + k;
        const double q = qs[iq];
        const double ga = J[((size_t)iq * (Lmax + 2) + Lmax + 1) * n_geo + g];
        double p = 1.0;
        for (int n = 0; n < lam; ++n) p *= q;
        double br = 0.0, bi = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            br = fma(p, w[m].x, br);
            bi = fma(p, w[m].y, bi);
            p *= q * q;
        }
        Bq[((size_t)k * nrows + row) * n_geo + g] = make_double2(br * ga, bi * ga);
    }
}

// Tile: 64 rows (state, lam mu) x 64 columns (L M) per workgroup, all
// geometries in chunks of 16, on the FP64 matrix cores
// (v_mfma_f64_16x16x4_f64: A = 16 rows x 4 geometries, B = 4 geometries x
// 16 columns; lane l holds A[l % 16][l / 16], B[l / 16][l % 16] and the
// results D[4 i + l / 16][l % 16], i = 0..3, as measured on the device).  Wave w owns the 16 rows 16 w .. 16 w + 15
// and all 4 column blocks; the complex product takes four real products
// (re re - im im, re im + im re).  The operands are staged in LDS as real and
// imaginary planes: thread t copies the row operand of row t / 4 at the four
// geometries 4 (t % 4) .. + 3 (formed per batch of radii by sph_b_kernel) and
// forms the column operand of column t % 64 at geometries t / 64 + 4 j
// (a = j_L Yt, Yt = 4 pi i^L Y* stored by the geometry kernel); the global
// loads of the next chunk are in flight while the current one is multiplied.
constexpr int kQRows = 64, kQCols = 64, kQK = 16;
constexpr int kQCB = kQCols / 16;   // column blocks per wave
typedef double sph_double4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void sph_q_kernel(const double* __restrict__ J, const double2* __restrict__ Yt,
                                                    const double2* __restrict__ Bq, int n_geo, int ns, int Lmax,
                                                    int iq0, double2* __restrict__ Q) {
    __shared__ double Br[kQRows][kQK + 1], Bi[kQRows][kQK + 1];
    __shared__ double Ar[kQK][kQCols + 1], Ai[kQK][kQCols + 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nrows = ns * kLam, ncols = (Lmax + 1) * (Lmax + 1);
    const int r0 = blockIdx.y * kQRows, c0 = blockIdx.x * kQCols;
    const int iq = iq0 + blockIdx.z;
    const double* Jq = J + (size_t)iq * (Lmax + 2) * n_geo;

    // row operand: row rb_ of the tile, geometries gq_ .. gq_ + 3 of a chunk
    const int rb_ = tid >> 2, gq_ = 4 * (tid & 3);
    const bool row_ok = r0 + rb_ < nrows;
    const double2* Brow = Bq + ((size_t)blockIdx.z * nrows + (row_ok ? r0 + rb_ : 0)) * n_geo;
    // column operand: column ca_ of the tile, geometries ga_ + 4 j of a chunk
    const int ca_ = tid & 63, ga_ = tid >> 6;
    const bool colA_ok = c0 + ca_ < ncols;
    const int colA = colA_ok ? c0 + ca_ : 0;
    const double* JL = Jq + (size_t)(int)sqrt((double)colA + 0.5) * n_geo;

    sph_double4 accR[kQCB], accI[kQCB];
#pragma unroll
    for (int cb = 0; cb < kQCB; ++cb) {
        accR[cb] = (sph_double4){0.0, 0.0, 0.0, 0.0};
        accI[cb] = (sph_double4){0.0, 0.0, 0.0, 0.0};
    }
    const int lr = lane & 15, lk = lane >> 4;
    const bool wave_rows = r0 + 16 * wave < nrows;   // wave-uniform
    // loads of a chunk: the row operand's run of 4 geometries, then Yt and
    // j_L at the column's four geometries; chunk g0 + kQK is loaded while the
    // matrix cores work on chunk g0.  The loads are unconditional, from
    // addresses clamped into the arrays, and the entries outside the problem
    // are zeroed when they are written to LDS (a conditional load joined with
    // a zero makes the compiler wait for it at once)
    double2 b[4], y[4];
    double jl[4];
    auto load_chunk = [&](int g0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = Brow[min(g0 + gq_ + j, n_geo - 1)];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int g = min(g0 + ga_ + 4 * j, n_geo - 1);
            y[j] = Yt[(size_t)g * ncols + colA];
            jl[j] = JL[g];
        }
    };
    load_chunk(0);
    for (int g0 = 0; g0 < n_geo; g0 += kQK) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool bok = row_ok && g0 + gq_ + j < n_geo;
            const bool aok = colA_ok && g0 + ga_ + 4 * j < n_geo;
            Br[rb_][gq_ + j] = bok ? b[j].x : 0.0;
            Bi[rb_][gq_ + j] = bok ? b[j].y : 0.0;
            Ar[ga_ + 4 * j][ca_] = aok ? jl[j] * y[j].x : 0.0;
            Ai[ga_ + 4 * j][ca_] = aok ? jl[j] * y[j].y : 0.0;
        }
        __syncthreads();
        if (g0 + kQK < n_geo) load_chunk(g0 + kQK);
        // a wave whose 16 rows all lie past the last row skips the products
        if (wave_rows) {
#pragma unroll
            for (int ks = 0; ks < kQK / 4; ++ks) {
                const double ar = Br[16 * wave + lr][4 * ks + lk], ai = Bi[16 * wave + lr][4 * ks + lk];
#pragma unroll
                for (int cb = 0; cb < kQCB; ++cb) {
                    const double br = Ar[4 * ks + lk][16 * cb + lr], bi = Ai[4 * ks + lk][16 * cb + lr];
                    accR[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, accR[cb], 0, 0, 0);
                    accR[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, accR[cb], 0, 0, 0);
                    accI[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, accI[cb], 0, 0, 0);
                    accI[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, accI[cb], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int cb = 0; cb < kQCB; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = r0 + 16 * wave + 4 * i + lk, col = c0 + 16 * cb + lr;
            if (r < nrows && col < ncols) Q[((size_t)iq * nrows + r) * ncols + col] = make_double2(accR[cb][i], accI[cb][i]);
        }
}

__global__ void sph_couple_kernel(const double2* __restrict__ Q, const double* __restrict__ gaunt, int ns, int lmax,
                                  int Lmax, int n_q, double2* __restrict__ R) {
    const int nl = (lmax + 1) * (lmax + 1), ncols = (Lmax + 1) * (Lmax + 1), nrows = ns * kLam;
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)ns * n_q * nl) return;
    const int lm = (int)(idx % nl);
    const long long r1 = idx / nl;
    const int iq = (int)(r1 % n_q), s = (int)(r1 / n_q);
    const int l = (int)sqrt((double)lm + 0.5), m = lm - l * l - l;
    double2 acc = make_double2(0.0, 0.0);
    for (int lam = 0; lam <= kSphMaxN; ++lam)
        for (int mu = -lam; mu <= lam; ++mu) {
            const int li = lam * lam + lam + mu;
            const double2* Qr = Q + ((size_t)iq * nrows + s * kLam + li) * ncols;
            const double* gr = gaunt + ((size_t)li * nl + lm) * kSphGauntJ;
            const int M = m - mu;
            for (int j = 0; j < kSphGauntJ; ++j) {
                const int L = abs(l - lam) + 2 * j;
                if (L > l + lam || abs(M) > L) continue;
                const double gv = gr[j];
                const double2 qv = Qr[L * L + L + M];
                acc.x += gv * qv.x;
                acc.y += gv * qv.y;
            }
        }
    R[((size_t)s * n_q + iq) * nl + lm] = acc;
}

// F^s(q, theta_i, m) = sum_{l >= |m|} R^s_lm(q) P~_l^m(cos theta_i), with
// Y_l^m = P~_l^m(cos theta) e^{i m phi} (P~ the normalised associated Legendre
// function with the Condon-Shortley phase; P~_l^{-m} = (-1)^m P~_l^m).
__global__ void sph_legendre_kernel(const double2* __restrict__ R, int ns, int lmax, int n_q, int n_theta,
                                    double2* __restrict__ F) {
    const int nm = 2 * lmax + 1, nl = (lmax + 1) * (lmax + 1);
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)n_q * n_theta * nm) return;
    const int mi = (int)(idx % nm);
    const long long r1 = idx / nm;
    const int it = (int)(r1 % n_theta), iq = (int)(r1 / n_theta);
    const int m = mi - lmax, am = abs(m);
    const double theta = n_theta > 1 ? M_PI * it / (n_theta - 1) : 0.0;
    double sn, cs;
    sincos(theta, &sn, &cs);
    double pmm = sqrt(1.0 / (4.0 * M_PI));
    for (int k = 1; k <= am; ++k) pmm *= -sqrt((2.0 * k + 1.0) / (2.0 * k)) * sn;
    const double sg = (m < 0 && (am & 1)) ? -1.0 : 1.0;
    for (int s = 0; s < ns; ++s) {
        const double2* Rs = R + ((size_t)s * n_q + iq) * nl;
        double2 acc = make_double2(0.0, 0.0);
        double p2 = 0.0, p1 = pmm;
        for (int l = am; l <= lmax; ++l) {
            double cur;
            if (l == am) {
                cur = pmm;
            } else if (l == am + 1) {
                cur = sqrt(2.0 * am + 3.0) * cs * pmm;
            } else {
                const double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)am * am));
                const double b = sqrt(((l - 1.0) * (l - 1.0) - (double)am * am) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
                cur = a * (cs * p1 - b * p2);
            }
            if (l > am) {
                p2 = p1;
                p1 = cur;
            }
            const double2 r = Rs[l * l + l + m];
            acc.x += sg * cur * r.x;
            acc.y += sg * cur * r.y;
        }
        F[(((size_t)s * n_q + iq) * n_theta + it) * nm + mi] = acc;
    }
}

// f^s(q, theta_i, phi_j) = sum_m F^s(q, theta_i, m) e^{i m phi_j}, phi_j = 2 pi j / n_phi.
__global__ void sph_phi_kernel(const double2* __restrict__ F, int ns, int lmax, int n_q, int n_theta, int n_phi,
                               float2* __restrict__ f, float* __restrict__ f2) {
    const int nm = 2 * lmax + 1;
    const long long npts = (long long)n_q * n_theta * n_phi;
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= npts) return;
    const int jp = (int)(idx % n_phi);
    const long long r1 = idx / n_phi;   // q, theta
    const double phi = 2.0 * M_PI * jp / n_phi;
    for (int s = 0; s < ns; ++s) {
        const double2* Fs = F + ((size_t)s * n_q * n_theta + r1) * nm;
        double2 acc = make_double2(0.0, 0.0);
        for (int mi = 0; mi < nm; ++mi) {
            double es, ec;
            sincos((mi - lmax) * phi, &es, &ec);
            const double2 v = Fs[mi];
            acc.x += v.x * ec - v.y * es;
            acc.y += v.x * es + v.y * ec;
        }
        const size_t o = (size_t)s * npts + idx;
        if (f) f[o] = make_float2((float)acc.x, (float)acc.y);
        if (f2) f2[o] = (float)(acc.x * acc.x + acc.y * acc.y);
    }
}

__global__ void sph_avg_kernel(const double2* __restrict__ R, int ns, int lmax, int n_q, double* __restrict__ avg) {
    const int nl = (lmax + 1) * (lmax + 1);
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ns * n_q) return;
    const double2* Rs = R + (size_t)idx * nl;
    double a = 0.0;
    for (int i = 0; i < nl; ++i) a += Rs[i].x * Rs[i].x + Rs[i].y * Rs[i].y;
    avg[idx] = a / (4.0 * M_PI);
}

}  // namespace

hipError_t launch_sph_geom(const SphGeom* geo, int n_geo, const VRowDev* rows, const int4* trow, const double* tp64,
                           int ns, const double2* theta, const int* uvw_idx, const int* nfirst, int n_nlm, int Lmax,
                           double4* gdat, double2* Yc, double2* W, hipStream_t st) {
    if (n_geo <= 0) return hipSuccess;
    hipLaunchKernelGGL(sph_geom_kernel, dim3((n_geo + 127) / 128), dim3(128), 0, st, geo, n_geo, rows, trow, tp64, ns,
                       theta, uvw_idx, nfirst, n_nlm, Lmax, gdat, Yc, W);
    return hipGetLastError();
}

hipError_t launch_sph_q(const double4* gdat, const double2* Yc, const double2* W, int n_geo, int ns, int Lmax,
                        const int* nlm_of, const double* qs, int n_q, double* J, double2* Bq, int nqb, double2* Q,
                        hipStream_t st) {
    if (nqb < 1) return hipErrorInvalidValue;
    const long long nb = (long long)n_q * n_geo;
    hipLaunchKernelGGL(sph_bessel_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, gdat, n_geo, Lmax, qs,
                       n_q, J);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nrows = ns * kLam, ncols = (Lmax + 1) * (Lmax + 1);
    if (nrows > 65535) return hipErrorInvalidValue;
    for (int iq0 = 0; iq0 < n_q; iq0 += nqb) {
        const int nk = std::min(nqb, n_q - iq0);
        hipLaunchKernelGGL(sph_b_kernel, dim3((n_geo + 255) / 256, nrows), dim3(256), 0, st, W, J, nlm_of, n_geo, ns,
                           Lmax, qs, iq0, nk, Bq);
        dim3 grid((ncols + kQCols - 1) / kQCols, (nrows + kQRows - 1) / kQRows, nk);
        hipLaunchKernelGGL(sph_q_kernel, grid, dim3(256), 0, st, J, Yc, Bq, n_geo, ns, Lmax, iq0, Q);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_sph_couple(const double2* Q, const double* gaunt, int ns, int lmax, int Lmax, int n_q, double2* R,
                             hipStream_t st) {
    const long long n = (long long)ns * n_q * (lmax + 1) * (lmax + 1);
    hipLaunchKernelGGL(sph_couple_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Q, gaunt, ns, lmax, Lmax,
                       n_q, R);
    return hipGetLastError();
}

hipError_t launch_sph_grid(const double2* R, int ns, int lmax, int n_q, int n_theta, int n_phi, double2* F, float2* f,
                           float* f2, hipStream_t st) {
    const long long n1 = (long long)n_q * n_theta * (2 * lmax + 1);
    hipLaunchKernelGGL(sph_legendre_kernel, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, R, ns, lmax, n_q,
                       n_theta, F);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long n2 = (long long)n_q * n_theta * n_phi;
    hipLaunchKernelGGL(sph_phi_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, F, ns, lmax, n_q, n_theta,
                       n_phi, f, f2);
    return hipGetLastError();
}

hipError_t launch_sph_avg(const double2* R, int ns, int lmax, int n_q, double* avg, hipStream_t st) {
    const int n = ns * n_q;
    hipLaunchKernelGGL(sph_avg_kernel, dim3((n + 255) / 256), dim3(256), 0, st, R, ns, lmax, n_q, avg);
    return hipGetLastError();
}

}  // namespace scff
