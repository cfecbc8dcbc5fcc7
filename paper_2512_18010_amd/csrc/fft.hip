// The FFT method (paper Sec. 3 and Sec. 5.2) on the device:
//
//   1. fft_pack_kernel /    transition weights as MFMA A operands:
//      fft_pack_bf_kernel   s_f c_mu c_nu (T_{mu nu} + T_{nu mu}) per unordered
//                           component pair (T_{mu mu} on the diagonal), FP32
//                           or split into BF16 halves;
//   2. fft_density_kernel   the transition density (eq. PhiTDM, AO form)
//                             Phi_s(r) = sum_mu phi_mu(r) sum_{nu >= mu} Tp_s(mu,nu) phi_nu(r)
//                           on a tile of up to 64 real-space points: the AO
//                           values of the tile are formed in LDS (FP64 and
//                           rounded once, or FP32 and split for the split-BF16
//                           contraction), Y_s(mu, r) = sum_nu Tp_s(mu,nu) phi_nu(r)
//                           runs on the matrix cores (rows mu of one state,
//                           k = nu, columns = points), and sum_mu phi_mu Y_s(mu)
//                           is folded per 16 rows.  Two states share one
//                           complex array (Phi_2b + i Phi_2b+1), so each FFT
//                           carries two.
//   3. fft_lines_kernel     radix-2 transforms of all lines of one axis of the
//                           complex arrays, a line group staged in LDS (eq.
//                           Falbega as three 1D passes);
//   4. fft_finish_kernel    separates the two states of each array
//                           (F_a = (Z_k + Z*_{-k})/2, F_b = (Z_k - Z*_{-k})/2i),
//                           orders the frequencies most negative first and
//                           applies the pixel volume and the corner phase:
//                           f_s(q) = V_pix e^{+i q.x_min} conj(F_s) (eq.
//                           fftABC for the conjugate array, eq. qabc);
//   5. fft_sum_kernel       the two sides of Parseval's identity (Sec. 7) from
//                           per-wave FP64 partial sums, in a fixed order.
#include <hip/hip_runtime.h>

#include "engine.h"

namespace scff {

typedef float fft_floatx4 __attribute__((ext_vector_type(4)));
typedef float fft_floatx2 __attribute__((ext_vector_type(2)));
typedef unsigned int fft_uintx4 __attribute__((ext_vector_type(4)));
typedef __bf16 fft_bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 fft_bf16x8 __attribute__((ext_vector_type(8)));

// Split-BF16 of one value: hi = RNE(v), lo = RNE(v - hi), each in the low
// half of a dword whose high half is zero.  v - hi is exact in FP32, so the
// BF16 dot product hi . (-1, -0) + v gives it in one instruction (-0, not +0:
// the compiler would encode (-1, +0) as the inline constant -1.0, which the
// instruction reads as the BF16 pair (+0, -1)).
__device__ inline void fft_split(float v, uint32_t& hi, uint32_t& lo) {
    const fft_bf16x2 h = __builtin_convertvector(fft_floatx2{v, 0.f}, fft_bf16x2);
    const float r = __builtin_amdgcn_fdot2_f32_bf16(h, fft_bf16x2{(__bf16)-1.0f, (__bf16)-0.0f}, v, false);
    hi = __builtin_bit_cast(uint32_t, h);
    lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(fft_floatx2{r, 0.f}, fft_bf16x2));
}
// The same in one dword: hi in the low half, lo in the high half.
__device__ inline uint32_t fft_split(float v) {
    uint32_t hi, lo;
    fft_split(v, hi, lo);
    return hi | (lo << 16);
}

// Primitives whose exponent argument alpha r^2 exceeds this are skipped (the
// paper's thresholding of negligible primitives): e^{-103} is below the
// smallest FP32 subnormal, so the rounded AO value is unchanged.
constexpr double kExpCut = 103.0;

// Grid points per density workgroup: one MFMA column block.

namespace {

__global__ void fft_pack_kernel(const double* __restrict__ T, const double* __restrict__ cnorm, int nbf, int ns,
                                int RB, int KS, double spin, float* __restrict__ Ap) {
    const long long total = (long long)ns * RB * KS * 64;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int lane = (int)(i & 63);
        long long r = i >> 6;
        const int ks = (int)(r % KS);
        r /= KS;
        const int rb = (int)(r % RB);
        const int s = (int)(r / RB);
        const int mu = 16 * rb + (lane & 15), nu = 4 * ks + (lane >> 4);
        double v = 0.0;
        if (mu < nbf && nu < nbf && mu <= nu) {
            const double* Ts = T + (size_t)s * nbf * nbf;
            const double t = mu == nu ? Ts[(size_t)mu * nbf + mu] : Ts[(size_t)mu * nbf + nu] + Ts[(size_t)nu * nbf + mu];
            v = spin * cnorm[mu] * cnorm[nu] * t;
        }
        Ap[i] = (float)v;
    }
}

// Split-BF16 A operands for the same weights.  Function group g holds
// nu = 16 g .. 16 g + 15; lane (row = lane % 16, kk = lane / 16) carries
// nu_j = 16 g + 4 kk + j, j < 4, as the words (hi(nu_0) | hi(nu_1) << 16,
// hi(nu_2) | hi(nu_3) << 16, lo(nu_0) | lo(nu_1) << 16, lo(nu_2) | lo(nu_3) << 16)
// in Ap[((s RB + rb) RB + g) 64 + lane].
__global__ void fft_pack_bf_kernel(const double* __restrict__ T, const double* __restrict__ cnorm, int nbf, int ns,
                                   int RB, double spin, uint4* __restrict__ Ap) {
    const long long total = (long long)ns * RB * RB * 64;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int lane = (int)(i & 63);
        long long r = i >> 6;
        const int g = (int)(r % RB);
        r /= RB;
        const int rb = (int)(r % RB);
        const int s = (int)(r / RB);
        const int mu = 16 * rb + (lane & 15);
        const double* Ts = T + (size_t)s * nbf * nbf;
        uint32_t w[4];
        for (int j = 0; j < 4; ++j) {
            const int nu = 16 * g + 4 * (lane >> 4) + j;
            double v = 0.0;
            if (mu < nbf && nu < nbf && mu <= nu) {
                const double tt =
                    mu == nu ? Ts[(size_t)mu * nbf + mu] : Ts[(size_t)mu * nbf + nu] + Ts[(size_t)nu * nbf + mu];
                v = spin * cnorm[mu] * cnorm[nu] * tt;
            }
            w[j] = fft_split((float)v);
        }
        Ap[i] = make_uint4((w[0] & 0xffffu) | (w[1] << 16), (w[2] & 0xffffu) | (w[3] << 16),
                           (w[0] >> 16) | (w[1] & 0xffff0000u), (w[2] >> 16) | (w[3] & 0xffff0000u));
    }
}

// e^{-x} for 0 <= x <= kExpCut in FP64, accurate to ~5e-9 relative (the
// value is rounded to FP32 afterwards): x = n ln2 + r with |r| <= ln2 / 2
// (ln2 in two parts, so r is exact to ~1e-16), e^{-r} by its Taylor
// polynomial of degree 7 (remainder r^8 / 8! < 5.2e-9), scaled by 2^{-n}.
__device__ __forceinline__ double fft_exp_neg(double x) {
    const double n = __builtin_rint(x * 1.4426950408889634);
    const double r = fma(n, 1.9082149292705877e-10, fma(n, 0.6931471803691238, -x));   // -(x - n ln2)
    double p = 1.0 / 5040.0;
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return __builtin_ldexp(p, -(int)n);
}

// AO values of one shell at one point before the contracted normalisation
// (c_mu is folded into the packed weights), handed to put(row, value) for
// each Cartesian component (row = bf0 + c).  F is double (the FP32
// contraction: values rounded once to FP32) or float (the split-BF16
// contraction, whose operands keep 16 significant bits: the offsets from the
// centre are formed in FP64 and rounded, the rest runs in FP32 with the
// hardware 2^x).
template <typename F, typename Put>
__device__ __forceinline__ void shell_values(const FftMol& m, int sh, double x, double y, double z, Put put) {
    const PrepShell S = m.shells[sh];
    const double* A = m.xyz + 3 * S.atom;
    const F dx = (F)(x - A[0]), dy = (F)(y - A[1]), dz = (F)(z - A[2]);
    const F r2 = dx * dx + dy * dy + dz * dz;
    // radial sums: sum_k d_k (product of 1D norms for the power pattern) e^{-alpha_k r^2}
    F ra = 0, rb = 0;   // l = 2: ra for xx-type, rb for xy-type; l < 2: ra only
    for (int k = 0; k < S.nprim; ++k) {
        const int o = S.off + k;
        const F ar = (F)m.exps[o] * r2;
        if (ar > (F)kExpCut) continue;
        F e;
        if constexpr (sizeof(F) == 8)
            e = (F)m.coefs[o] * fft_exp_neg(ar);
        else
            e = (F)m.coefs[o] * __builtin_amdgcn_exp2f(ar * -1.44269504f);
        const F n0 = (F)m.n1d[3 * o], n1 = (F)m.n1d[3 * o + 1], n2 = (F)m.n1d[3 * o + 2];
        if (S.l == 0) {
            ra += e * (n0 * n0 * n0);
        } else if (S.l == 1) {
            ra += e * (n1 * n0 * n0);
        } else {
            ra += e * (n2 * n0 * n0);
            rb += e * (n1 * n1 * n0);
        }
    }
    const int b0 = m.bf0[sh];
    if (S.l == 0) {
        put(b0, ra);
    } else if (S.l == 1) {
        put(b0, dx * ra);
        put(b0 + 1, dy * ra);
        put(b0 + 2, dz * ra);
    } else {
        put(b0, dx * dx * ra);
        put(b0 + 1, dx * dy * rb);
        put(b0 + 2, dx * dz * rb);
        put(b0 + 3, dy * dy * ra);
        put(b0 + 4, dy * dz * rb);
        put(b0 + 5, dz * dz * ra);
    }
}

// LDS bytes of a density workgroup: the AO block of nbf_pad rows x 16 CB
// points (4 bytes per value in either layout) and two buffers of 4 x 16 CB
// FP64 partial densities.
__host__ __device__ constexpr size_t fft_lds_bytes(int nbf_pad, int cb) {
    return (size_t)cb * (64 * (size_t)nbf_pad + 1024);
}

// One workgroup (4 waves) per tile of NP = 16 CB consecutive grid points
// (flattened [ix][iy][iz], z fastest; column c = 16 cb + col of the tile).
//
// AO phase: a lane evaluates one shell at one point (64 / NP shells per wave
// step; with NP = 64 every lane of a wave takes the same shell, so its data
// are scalar loads), FP64, rounded into the LDS block:
//   FP32  phi(r, c) at float index r NP + col CB + cb, so that a lane reads the
//         CB values of its column in one ds_read (b32 / b64 / b128) and a
//         quarter wave reads one contiguous run (no bank conflicts);
//   BF    split halves as the B operands of v_mfma_f32_16x16x32_bf16: the
//         uint4 entry ((g 4 + kk) CB + cb) 16 + col holds rows r_j = 16 g +
//         4 kk + j (j < 4) of column c as (hi(r_0) | hi(r_1) << 16, hi(r_2) |
//         hi(r_3) << 16, lo(r_0) | lo(r_1) << 16, lo(r_2) | lo(r_3) << 16).
//         A lane (kk, col) takes it as the 8 k-items of one MFMA (no operand
//         copies), and the same entry holds the rows 16 rb + 4 kk + i that
//         the lane folds after row block rb.
// Split-BF16 products per function group and column block: MFMA 1 with
// A = (W hi, W hi) gives hi*hi + hi*lo over the items, MFMA 2 with
// A = (W lo, 0) gives lo*hi.
//
// Contraction: wave w takes row blocks rb of 16 functions in a snake order
// (0 1 2 3 3 2 1 0 ...), which evens out the triangle's rows; per row block
// the k-steps from the diagonal block on, with the A operands of the next
// k-steps loaded while the current ones run and each A operand used by CB
// MFMAs.  The 16-row block is folded with its AO values, the four waves'
// partial densities of a group of states are summed through LDS and wave 0
// writes the tile.
template <bool BF, int CB>
__global__ __launch_bounds__(256) void fft_density_kernel(FftMol m, const void* __restrict__ Av, int nbf_pad, int ns,
                                                          int RB, int KS, int3 n, double3 x0, double3 h,
                                                          long long npts, float* __restrict__ Z,
                                                          float* __restrict__ phi_out, double* __restrict__ psum) {
    extern __shared__ __align__(16) float fft_lds[];
    constexpr int NP = 16 * CB;
    constexpr int NCH = CB == 1 ? 2 : CB;   // independent MFMA accumulator chains
    const int tid = threadIdx.x, lane = tid & 63;
    // wave-uniform: the row-block loop and the A-operand addresses stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const long long p0 = (long long)blockIdx.x * NP;
    float* ph = fft_lds;
    uint32_t* pu = reinterpret_cast<uint32_t*>(fft_lds);
    unsigned short* ps16 = reinterpret_cast<unsigned short*>(fft_lds);
    double* red = reinterpret_cast<double*>(fft_lds + (size_t)nbf_pad * NP);

    for (int i = tid; i < nbf_pad * NP; i += 256) pu[i] = 0u;
    __syncthreads();
    {
        constexpr int SPI = 64 / NP;   // shells per wave step
        const int p = lane % NP;
        const long long g = p0 + p;
        const int iz = (int)(g % n.z);
        const long long r1 = g / n.z;
        const int iy = (int)(r1 % n.y), ix = (int)(r1 / n.y);
        const double x = x0.x + ix * h.x, y = x0.y + iy * h.y, z = x0.z + iz * h.z;
        const int col = p & 15, cb = p >> 4;
        auto put = [&](int r, auto v) {
            if constexpr (BF) {
                uint32_t hi, lo;
                fft_split((float)v, hi, lo);
                const int i = r & 3;
                // dword of the hi half; the lo half is two dwords on
                const int wd = ((((r >> 4) * 4 + ((r >> 2) & 3)) * CB + cb) * 16 + col) * 4 + (i >> 1);
                ps16[2 * wd + (i & 1)] = (unsigned short)hi;
                ps16[2 * wd + 4 + (i & 1)] = (unsigned short)lo;
            } else {
                ph[r * NP + col * CB + cb] = (float)v;
            }
        };
        for (int sh0 = wave * SPI; sh0 < m.n_shells; sh0 += 4 * SPI) {
            const int sh = sh0 + lane / NP;
            if (sh < m.n_shells && g < npts) shell_values<std::conditional_t<BF, float, double>>(m, sh, x, y, z, put);
        }
    }

    const int kk = lane >> 4, col = lane & 15;
    // the AO values of rows 16 rb + 4 kk + i (i < 4) at this lane's CB columns,
    // v[i][cb] (in the split form hi + lo, summed in FP32: within 2^-24 of the
    // split value, far below the split's own 2^-16)
    using FV = std::conditional_t<BF, float, double>;
    auto phi_rows = [&](int rb, FV (&v)[4][CB]) {
        if constexpr (BF) {
#pragma unroll
            for (int q = 0; q < CB; ++q) {
                const uint4 e = reinterpret_cast<const uint4*>(pu)[((rb * 4 + kk) * CB + q) * 16 + col];
                v[0][q] = __uint_as_float(e.x << 16) + __uint_as_float(e.z << 16);
                v[1][q] = __uint_as_float(e.x & 0xffff0000u) + __uint_as_float(e.z & 0xffff0000u);
                v[2][q] = __uint_as_float(e.y << 16) + __uint_as_float(e.w << 16);
                v[3][q] = __uint_as_float(e.y & 0xffff0000u) + __uint_as_float(e.w & 0xffff0000u);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float* q = ph + (16 * rb + 4 * kk + i) * NP + col * CB;
                if constexpr (CB == 1) {
                    v[i][0] = q[0];
                } else if constexpr (CB == 2) {
                    const float2 e = *reinterpret_cast<const float2*>(q);
                    v[i][0] = e.x;
                    v[i][1] = e.y;
                } else {
                    const float4 e = *reinterpret_cast<const float4*>(q);
                    v[i][0] = e.x;
                    v[i][1] = e.y;
                    v[i][2] = e.z;
                    v[i][3] = e.w;
                }
            }
        }
    };
    __syncthreads();

    // one k-step (FP32: functions 4k .. 4k+3) or k-group (BF: 8t .. 8t+7) of
    // row block rb for all CB column blocks
    auto kstep = [&](auto a, int k, int par, fft_floatx4 (&c)[NCH]) {
        if constexpr (BF) {
            const fft_bf16x8 A1 = __builtin_bit_cast(fft_bf16x8, fft_uintx4{a.x, a.y, a.x, a.y});
            const fft_bf16x8 A2 = __builtin_bit_cast(fft_bf16x8, fft_uintx4{a.z, a.w, 0u, 0u});
            fft_bf16x8 B[CB];
#pragma unroll
            for (int q = 0; q < CB; ++q) {
                const uint4 e = reinterpret_cast<const uint4*>(pu)[((k * 4 + kk) * CB + q) * 16 + col];
                B[q] = __builtin_bit_cast(fft_bf16x8, fft_uintx4{e.x, e.y, e.z, e.w});
            }
            // the two products of a column block go to different chains (CB = 1)
            // or are CB instructions apart
#pragma unroll
            for (int q = 0; q < CB; ++q) c[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B[q], c[q], 0, 0, 0);
#pragma unroll
            for (int q = 0; q < CB; ++q)
                c[CB == 1 ? 1 : q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2, B[q], c[CB == 1 ? 1 : q], 0, 0, 0);
        } else {
            const float* q = ph + (4 * k + kk) * NP + col * CB;
            if constexpr (CB == 1) {
                c[par] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, q[0], c[par], 0, 0, 0);
            } else if constexpr (CB == 2) {
                const float2 e = *reinterpret_cast<const float2*>(q);
                c[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, e.x, c[0], 0, 0, 0);
                c[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, e.y, c[1], 0, 0, 0);
            } else {
                const float4 e = *reinterpret_cast<const float4*>(q);
                c[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, e.x, c[0], 0, 0, 0);
                c[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, e.y, c[1], 0, 0, 0);
                c[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, e.z, c[2], 0, 0, 0);
                c[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, e.w, c[3], 0, 0, 0);
            }
        }
    };

    // the k-steps k0 .. k0 + nk - 1 of one row block (nk a multiple of GS, at
    // least GS).  The main loop runs whole blocks of 2 PD k-steps with no exit
    // inside, the A operands of the next PD k-steps loaded while the current
    // PD run (an exit between a load and its use lets the compiler sink the
    // load to the use, which then waits for it); the last 0 .. 2 PD - GS
    // k-steps run in a guarded tail.  Loads past the row block read the next
    // block or the array's slack and are not used.
    constexpr int GS = BF ? 1 : 4;
    constexpr int PD = BF ? 4 : 8;   // k-steps per register set (prefetch depth)
    auto run_row = [&](const auto* ap, auto (&A0)[PD], auto (&A1)[PD], int k0, int nk, fft_floatx4 (&c)[NCH]) {
#pragma unroll
        for (int j = 0; j < PD; ++j) A0[j] = ap[j * 64];
        int t = 0;
        for (; t + 2 * PD <= nk; t += 2 * PD) {
            const auto* q = ap + (size_t)t * 64;
#pragma unroll
            for (int j = 0; j < PD; ++j) A1[j] = q[(PD + j) * 64];
#pragma unroll
            for (int j = 0; j < PD; ++j) kstep(A0[j], k0 + t + j, j & 1, c);
#pragma unroll
            for (int j = 0; j < PD; ++j) A0[j] = q[(2 * PD + j) * 64];
#pragma unroll
            for (int j = 0; j < PD; ++j) kstep(A1[j], k0 + t + PD + j, j & 1, c);
        }
        const int r = nk - t;   // wave-uniform
        if (r > 0) {
            const auto* q = ap + (size_t)t * 64;
#pragma unroll
            for (int j = 0; j < PD; ++j) A1[j] = q[(PD + j) * 64];
#pragma unroll
            for (int j = 0; j < PD; j += GS) {
                if (j >= r) return;
#pragma unroll
                for (int i = 0; i < GS; ++i) kstep(A0[j + i], k0 + t + j + i, (j + i) & 1, c);
            }
#pragma unroll
            for (int j = 0; j < PD; j += GS) {
                if (PD + j >= r) return;
#pragma unroll
                for (int i = 0; i < GS; ++i) kstep(A1[j + i], k0 + t + PD + j + i, (j + i) & 1, c);
            }
        }
    };

    // States in groups of SG: the AO values of a row block are formed once per
    // group, and the four waves' partial densities of the group meet in one
    // LDS slot (two barriers per group).  The fold over a wave's row blocks is
    // FP64 for the FP32 contraction and FP32 for split-BF16 (whose products
    // carry 16 significant bits); the slot holds SG x 4 x NP of them, within
    // the 64 NP bytes set aside.
    constexpr int SG = 2;
    FV* rd = reinterpret_cast<FV*>(red);
    for (int s0 = 0; s0 < ns; s0 += SG) {
        FV acc[SG][CB];
#pragma unroll
        for (int si = 0; si < SG; ++si)
#pragma unroll
            for (int q = 0; q < CB; ++q) acc[si][q] = 0;
        for (int i4 = 0; i4 < RB; i4 += 4) {
            // snake order: blocks i4 .. i4+3 go to waves 0..3, then 3..0
            const int rb = i4 + (((i4 >> 2) & 1) ? 3 - wave : wave);
            if (rb >= RB) continue;
            // lane (kk, col) holds rows 16 rb + 4 kk + i of its columns
            FV v[4][CB];
            phi_rows(rb, v);
#pragma unroll
            for (int si = 0; si < SG; ++si) {
                const int s = s0 + si;
                if (s >= ns) break;
                fft_floatx4 c[NCH];
#pragma unroll
                for (int q = 0; q < NCH; ++q) c[q] = fft_floatx4{0.f, 0.f, 0.f, 0.f};
                if constexpr (BF) {
                    const int k0 = rb, nk = RB - k0;
                    const uint4* ap =
                        reinterpret_cast<const uint4*>(Av) + ((size_t)(s * RB + rb) * RB + k0) * 64 + lane;
                    uint4 A0[PD], A1[PD];
                    run_row(ap, A0, A1, k0, nk, c);
                } else {
                    const int k0 = 4 * rb, nk = KS - k0;
                    const float* ap =
                        reinterpret_cast<const float*>(Av) + ((size_t)(s * RB + rb) * KS + k0) * 64 + lane;
                    float A0[PD], A1[PD];
                    run_row(ap, A0, A1, k0, nk, c);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int q = 0; q < CB; ++q) {
                        const float y = CB == 1 ? c[0][i] + c[1][i] : c[q][i];
                        acc[si][q] += v[i][q] * (FV)y;
                    }
            }
        }
#pragma unroll
        for (int si = 0; si < SG; ++si)
#pragma unroll
            for (int q = 0; q < CB; ++q) {
                FV a = acc[si][q];
                a += __shfl_xor(a, 16);
                a += __shfl_xor(a, 32);
                if (lane < 16) rd[(si * 4 + wave) * NP + q * 16 + lane] = a;
            }
        __syncthreads();
        if (wave == 0) {
            const long long g = p0 + lane;
            const bool valid = lane < NP && g < npts;
#pragma unroll
            for (int si = 0; si < SG; ++si) {
                const int s = s0 + si;
                if (s >= ns) break;
                const FV* r4 = rd + si * 4 * NP;
                double d = 0.0;
                if (lane < NP) d = (double)r4[lane] + (double)r4[NP + lane] + (double)r4[2 * NP + lane] + (double)r4[3 * NP + lane];
                if (valid) {
                    const float v = (float)d;
                    float* zp = Z + ((size_t)(s >> 1) * npts + g) * 2;
                    zp[s & 1] = v;
                    if ((ns & 1) && s == ns - 1) zp[1] = 0.f;
                    if (phi_out) phi_out[(size_t)s * npts + g] = v;
                }
                double q = valid ? d * d : 0.0;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) q += __shfl_xor(q, o);
                if (psum && lane == 0) psum[(size_t)s * gridDim.x + blockIdx.x] = q;
            }
        }
        __syncthreads();
    }
}

// Lines of one axis of the complex arrays Z[nb][nx][ny][nz]: a workgroup
// transforms M lines of length N in LDS (radix-2, decimation in time on
// bit-reversed input), with twiddles e^{-2 pi i k / N} built in FP64 and
// rounded.  Along z the M lines are consecutive rows; along y and x they are
// M consecutive z, so every load and store touches contiguous runs.
__global__ __launch_bounds__(256) void fft_lines_kernel(float2* __restrict__ Z, int axis, int3 n, int nb, int M,
                                                        long long lines) {
    extern __shared__ __align__(16) float fft_lds[];
    const int N = axis == 0 ? n.x : axis == 1 ? n.y : n.z;
    const int logN = 31 - __clz(N);
    float2* buf = reinterpret_cast<float2*>(fft_lds);
    float2* tw = buf + (size_t)M * N;
    for (int k = threadIdx.x; k < N / 2; k += blockDim.x) {
        double sn, cs;
        sincospi(-2.0 * k / N, &sn, &cs);
        tw[k] = make_float2((float)cs, (float)sn);
    }
    const long long plane = (long long)n.y * n.z, vol = (long long)n.x * plane;
    const long long gidx = blockIdx.x;
    long long base, es, ls;
    int mcount = M;
    if (axis == 2) {
        base = gidx * M * N;
        es = 1;
        ls = N;
        const long long left = lines - gidx * M;
        if (left < M) mcount = (int)left;
    } else {
        const int zb = n.z / M;
        const int z0 = (int)(gidx % zb) * M;
        const long long r = gidx / zb;
        if (axis == 1) {
            const int x = (int)(r % n.x);
            const long long b = r / n.x;
            base = b * vol + (long long)x * plane + z0;
            es = n.z;
        } else {
            const int y = (int)(r % n.y);
            const long long b = r / n.y;
            base = b * vol + (long long)y * n.z + z0;
            es = plane;
        }
        ls = 1;
    }
    (void)nb;
    const int tot = mcount * N;
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        int mm, k;
        if (axis == 2) {
            mm = i / N;
            k = i - mm * N;
        } else {
            k = i / mcount;
            mm = i - k * mcount;
        }
        const float2 v = Z[base + mm * ls + k * es];
        buf[mm * N + (int)(__brev((unsigned)k) >> (32 - logN))] = v;
    }
    __syncthreads();
    const int hN = N / 2;
    for (int len = 2; len <= N; len <<= 1) {
        const int half = len >> 1, tstep = N / len;
        for (int j = threadIdx.x; j < mcount * hN; j += blockDim.x) {
            const int mm = j / hN, r = j - mm * hN;
            const int grp = r / half, pos = r - grp * half;
            const int i0 = mm * N + grp * len + pos, i1 = i0 + half;
            const float2 w = tw[pos * tstep];
            const float2 a = buf[i0], b = buf[i1];
            const float tr = w.x * b.x - w.y * b.y, ti = w.x * b.y + w.y * b.x;
            buf[i0] = make_float2(a.x + tr, a.y + ti);
            buf[i1] = make_float2(a.x - tr, a.y - ti);
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        int mm, k;
        if (axis == 2) {
            mm = i / N;
            k = i - mm * N;
        } else {
            k = i / mcount;
            mm = i - k * mcount;
        }
        Z[base + mm * ls + k * es] = buf[mm * N + k];
    }
}

// One thread per output point (i, j, k) of every state: q_a = 2 pi (i_a - n_a/2) / L_a.
__global__ __launch_bounds__(256) void fft_finish_kernel(const float2* __restrict__ Z, int3 n, int ns, double vpix,
                                                         double3 u, long long npts, float2* __restrict__ f,
                                                         float* __restrict__ f2, double* __restrict__ psum) {
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const bool valid = idx < npts;
    const int lane = threadIdx.x & 63;
    const long long wv = idx >> 6;   // global wave index
    const long long nwv = (npts + 63) >> 6;
    long long src = 0, mir = 0;
    double cs = 1.0, sn = 0.0;
    if (valid) {
        const int k = (int)(idx % n.z);
        const long long r1 = idx / n.z;
        const int j = (int)(r1 % n.y), i = (int)(r1 / n.y);
        const int ai = i - n.x / 2, aj = j - n.y / 2, ak = k - n.z / 2;
        const int si = (i + n.x / 2) & (n.x - 1), sj = (j + n.y / 2) & (n.y - 1), sk = (k + n.z / 2) & (n.z - 1);
        const int mi = (n.x - si) & (n.x - 1), mj = (n.y - sj) & (n.y - 1), mk = (n.z - sk) & (n.z - 1);
        src = ((long long)si * n.y + sj) * n.z + sk;
        mir = ((long long)mi * n.y + mj) * n.z + mk;
        // q.x_min / (2 pi) in turns, reduced to [-1/2, 1/2], in FP64
        double t = ai * u.x + aj * u.y + ak * u.z;
        t -= rint(t);
        sincospi(2.0 * t, &sn, &cs);
    }
    for (int s = 0; s < ns; ++s) {
        double a2 = 0.0;
        if (valid) {
            const float2 zs = Z[(size_t)(s >> 1) * npts + src];
            const float2 zm = Z[(size_t)(s >> 1) * npts + mir];
            double fr, fi;   // F_s
            if ((s & 1) == 0) {
                fr = 0.5 * ((double)zs.x + (double)zm.x);
                fi = 0.5 * ((double)zs.y - (double)zm.y);
            } else {
                fr = 0.5 * ((double)zs.y + (double)zm.y);
                fi = -0.5 * ((double)zs.x - (double)zm.x);
            }
            // f = V_pix e^{i theta} conj(F)
            const double vr = vpix * (cs * fr + sn * fi), vi = vpix * (sn * fr - cs * fi);
            a2 = vr * vr + vi * vi;
            const size_t o = (size_t)s * npts + idx;
            if (f) f[o] = make_float2((float)vr, (float)vi);
            if (f2) f2[o] = (float)a2;
        }
        if (psum) {
            for (int d = 1; d < 64; d <<= 1) a2 += __shfl_xor(a2, d);
            if (lane == 0 && wv < nwv) psum[(size_t)s * nwv + wv] = a2;
        }
    }
}

// out[s * stride] = sum of part[s][0..n) in a fixed order (one workgroup per state).
__global__ __launch_bounds__(256) void fft_sum_kernel(const double* __restrict__ part, long long n, double scale,
                                                      double* __restrict__ out, int stride) {
    __shared__ double sm[256];
    const int s = blockIdx.x;
    double a = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) a += part[(size_t)s * n + i];
    sm[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)s * stride] = scale * sm[0];
}

}  // namespace

hipError_t launch_fft_pack(int precision, const double* T, const double* cnorm, int nbf, int ns, int RB, int KS,
                           double spin, void* Ap, hipStream_t st) {
    const long long total = (long long)ns * RB * (precision == SCFF_BF16X3 ? RB : KS) * 64;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 65536);
    if (precision == SCFF_BF16X3)
        hipLaunchKernelGGL(fft_pack_bf_kernel, dim3(blocks), dim3(256), 0, st, T, cnorm, nbf, ns, RB, spin,
                           (uint4*)Ap);
    else
        hipLaunchKernelGGL(fft_pack_kernel, dim3(blocks), dim3(256), 0, st, T, cnorm, nbf, ns, RB, KS, spin,
                           (float*)Ap);
    return hipGetLastError();
}

int fft_density_cb(int nbf_pad, size_t lds_limit) {
    // the widest tile whose block stays within 64 KiB (several workgroups per
    // CU); 16-point tiles up to the device limit for the largest bases
    for (int cb : {4, 2})
        if (fft_lds_bytes(nbf_pad, cb) <= std::min<size_t>(lds_limit, 64u << 10)) return cb;
    return fft_lds_bytes(nbf_pad, 1) <= lds_limit ? 1 : 0;
}

hipError_t launch_fft_density(int precision, const FftMol& m, const void* Ap, int nbf_pad, int ns, int RB, int KS,
                              const int n[3], const double x0[3], const double h[3], float* Z, float* phi, double* psum,
                              size_t lds_limit, long long* n_part, hipStream_t st) {
    const long long npts = (long long)n[0] * n[1] * n[2];
    const int cb = fft_density_cb(nbf_pad, lds_limit);
    if (cb == 0 || nbf_pad % 16 || KS * 4 != nbf_pad || RB * 16 != nbf_pad) return hipErrorInvalidValue;
    const size_t lds = fft_lds_bytes(nbf_pad, cb);
    const long long tiles = (npts + 16 * cb - 1) / (16 * cb);
    if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
    *n_part = tiles;
    const bool bf = precision == SCFF_BF16X3;
    const void* fns[2][3] = {{(const void*)fft_density_kernel<false, 1>, (const void*)fft_density_kernel<false, 2>,
                              (const void*)fft_density_kernel<false, 4>},
                             {(const void*)fft_density_kernel<true, 1>, (const void*)fft_density_kernel<true, 2>,
                              (const void*)fft_density_kernel<true, 4>}};
    const int ci = cb == 4 ? 2 : cb - 1;
    if (lds > 65536) {
        // dynamic LDS beyond 64 KiB per workgroup must be allowed explicitly
        const hipError_t e = hipFuncSetAttribute(fns[bf][ci], hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int3 nn = make_int3(n[0], n[1], n[2]);
    const double3 xx = make_double3(x0[0], x0[1], x0[2]), hh = make_double3(h[0], h[1], h[2]);
    const dim3 grid((unsigned)tiles), block(256);
#define SCFF_FFT_DENSITY(B, C)                                                                                  \
    hipLaunchKernelGGL((fft_density_kernel<B, C>), grid, block, lds, st, m, Ap, nbf_pad, ns, RB, KS, nn, xx, hh, \
                       npts, Z, phi, psum)
    if (bf) {
        if (cb == 4) SCFF_FFT_DENSITY(true, 4);
        else if (cb == 2) SCFF_FFT_DENSITY(true, 2);
        else SCFF_FFT_DENSITY(true, 1);
    } else {
        if (cb == 4) SCFF_FFT_DENSITY(false, 4);
        else if (cb == 2) SCFF_FFT_DENSITY(false, 2);
        else SCFF_FFT_DENSITY(false, 1);
    }
#undef SCFF_FFT_DENSITY
    return hipGetLastError();
}

hipError_t launch_fft_lines(float2* Z, int nb, const int n[3], hipStream_t st) {
    const int3 nn = make_int3(n[0], n[1], n[2]);
    for (int axis = 2; axis >= 0; --axis) {
        const int N = n[axis];
        if (N < 2) continue;
        long long lines;
        int M;
        long long groups;
        if (axis == 2) {
            lines = (long long)nb * n[0] * n[1];
            M = std::max(1, 4096 / N);
            groups = (lines + M - 1) / M;
        } else {
            M = std::min(std::min(16, n[2]), std::max(1, 4096 / N));
            lines = (long long)nb * n[0] * n[1] * n[2] / N;
            groups = lines / M;
        }
        if (groups > 0x7fffffffLL) return hipErrorInvalidValue;
        const size_t lds = ((size_t)M * N + N / 2) * sizeof(float2);
        hipLaunchKernelGGL(fft_lines_kernel, dim3((unsigned)groups), dim3(256), lds, st, Z, axis, nn, nb, M, lines);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fft_finish(const float2* Z, const int n[3], int ns, double vpix, const double u[3], float2* f,
                             float* f2, double* psum, long long* n_part, hipStream_t st) {
    const long long npts = (long long)n[0] * n[1] * n[2];
    const long long blocks = (npts + 255) / 256;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    *n_part = (npts + 63) / 64;
    hipLaunchKernelGGL(fft_finish_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Z, make_int3(n[0], n[1], n[2]),
                       ns, vpix, make_double3(u[0], u[1], u[2]), npts, f, f2, psum);
    return hipGetLastError();
}

hipError_t launch_fft_sum(const double* part, int ns, long long n, double scale, double* out, int stride,
                          hipStream_t st) {
    hipLaunchKernelGGL(fft_sum_kernel, dim3(ns), dim3(256), 0, st, part, n, scale, out, stride);
    return hipGetLastError();
}

}  // namespace scff
