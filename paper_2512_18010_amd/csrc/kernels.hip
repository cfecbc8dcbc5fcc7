// Device kernels of the Cartesian form-factor engine (gfx950 / CDNA4).
//
// Hot path (paper Sec. 4 eq. CartesianMethod, Sec. 5.3):
//
//   f_s(qx,qy,qz) = sum_k Tp(s,k) G(k,q),
//   G(k,q)        = sum_{t in terms(k)} Vx_t(qx) Vy_t(qy) Vz_t(qz),
//
// where k runs over unique component pairs (mu <= nu), t over their kept
// primitive-pair terms, and V_t^a are the 1D V-tensors of eq.
// CartesianVector in monomial form (eq. Ccoefficients).
//
//  * vtable_kernel: the 1D tables V[row][n] for every grid value of each
//    axis (O(rows x N) work, a precompute next to the O(R x N^3) bulk).  They
//    are evaluated in FP64 (phase q*P with range reduction, Gaussian,
//    polynomial) and rounded once to FP32: the polynomial can cancel, and
//    FP32 evaluation would leave errors proportional to its bound rather
//    than to its value.
//  * grid_kernel: one workgroup per q-tile of 4 x 8 lines (qx,qy) x
//    (4*QZL) values of qz.  Per chunk of 8-32 component pairs the tile's
//    W = Vx*Vy (per line) and Vz (per qz) slices are staged in LDS; every
//    lane then forms G for 2 lines x QZL qz values of one component pair on
//    the VALU and feeds it, still in registers, to the matrix cores.  FP32:
//    v_mfma_f32_16x16x4_f32 (A = Tp, 16 states x 4 pairs), with the FP32
//    MFMA sums of every 32 pairs folded into FP64 totals, which bounds the
//    rounding error of the long, cancelling pair sum.  Split-BF16 (template
//    flag BF): G and Tp as hi + lo BF16 halves, lo*hi + hi*hi + hi*lo of one
//    unit (8 pairs) in one v_mfma_f32_16x16x32_bf16 with FP32 accumulation.
//  * points_kernel: the same sum at arbitrary points (VALU only), V
//    evaluated on the fly.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "engine.h"
#include "vrow.h"

namespace scff {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Two FP32 values -> two round-to-nearest-even BF16 in one dword (a in the low half).
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(floatx2{a, b}, bf16x2));
}
// Split-BF16 of two values: hi = RNE(g), lo = RNE(g - hi).  g - hi is exact
// in FP32 (hi is a multiple of g's FP32 ulp and |g - hi| needs at most 16
// significant bits), so any correctly rounded evaluation of it gives the same
// value; a BF16 dot product hi . (-1, -0) + g forms it in one instruction,
// without unpacking hi.  The weights carry -0 rather than +0 in the other
// half: the compiler encodes (-1, +0) as the inline constant -1.0, which the
// instruction reads as the FP32 pattern of -1.0, i.e. the BF16 pair (+0, -1);
// (-1, -0) and (-0, -1) have no inline form and go as literals.
__device__ __forceinline__ void split_bf16(float g0, float g1, uint32_t& hi, uint32_t& lo) {
    const bf16x2 h = __builtin_convertvector(floatx2{g0, g1}, bf16x2);
    const float l0 = __builtin_amdgcn_fdot2_f32_bf16(h, bf16x2{(__bf16)-1.0f, (__bf16)-0.0f}, g0, false);
    const float l1 = __builtin_amdgcn_fdot2_f32_bf16(h, bf16x2{(__bf16)-0.0f, (__bf16)-1.0f}, g1, false);
    hi = __builtin_bit_cast(uint32_t, h);
    lo = pack_bf16(l0, l1);
}
// Eight BF16 k-items of a 16x16x32 operand, two per dword (low half first).
__device__ __forceinline__ bf16x8 bf16x8_of(uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1) {
    return __builtin_bit_cast(bf16x8, uintx4{a0, a1, b0, b1});
}

constexpr int kPointFoldUnits = 4;   // points kernel: units (32 pairs) per FP32 block sum

// ---------------------------------------------------------------- 1D tables

__device__ __forceinline__ float2 eval_row(const VRowDev& r, double q) {
    const double2 v = eval_row_fp64(r, q);
    return make_float2((float)v.x, (float)v.y);
}

__global__ void vtable_kernel(const VRowDev* __restrict__ rows, int nrows, int vstride,
                              int3 n, double3 qmin, double3 dq, float2* __restrict__ V) {
    const long long tot = (long long)nrows * vstride;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < tot;
         i += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(i / vstride);
        const int j = (int)(i - (long long)r * vstride);
        const VRowDev row = rows[r];
        const int ax = row.axis;
        const int na = ax == 0 ? n.x : (ax == 1 ? n.y : n.z);
        if (j >= na) {
            V[i] = make_float2(0.f, 0.f);
            continue;
        }
        const double q0 = ax == 0 ? qmin.x : (ax == 1 ? qmin.y : qmin.z);
        const double d = ax == 0 ? dq.x : (ax == 1 ? dq.y : dq.z);
        V[i] = eval_row(row, q0 + d * (double)j);
    }
}

// ---------------------------------------------------------------- grid kernel
//
// Workgroup = NW waves (4 or 8), tile = 4 qx x 8 qy lines x TZ qz
// (TZ = 4*QZL per q_x line of waves; 8 waves put two waves on each q_x line,
// one per half of the q_z range, so the chunk staging serves twice the q
// values).
// The packed pairs come in units of 8 component pairs with npp terms each
// (npp <= 9); a chunk is a run of 1..4 consecutive units with the same npp
// and at most 72 terms (up to 32 pairs when npp <= 2).  Per chunk, for every
// term t (index ptl = (unit*8 + pair)*npp + term):
//   raw slices  Vx[t][4], Vy[t][8], Vz[t][TZ]   global -> LDS by direct DMA
//   W[t][line] = Vx * Vy                        cooperative, in LDS
// plus the chunk's packed weights Tp[pairs][16*SB] (DMA as well).  The raw
// slices and Tp are double-buffered: the DMA for chunk c+1 is issued at the
// start of chunk c and completes under chunk c's W phase and main loop; the
// row ids it needs were loaded one chunk earlier.  With one state block (SB =
// 1) V^x and V^y, which only the W phase reads, have a single buffer of
// their own, refilled for chunk c+1 right after chunk c's W phase: 50 KB of
// LDS per workgroup instead of 60, which lets the split-BF16 variants (156-160
// VGPRs) hold three workgroups per CU; the variants with two state blocks
// keep all slices of a term in one double-buffered row (their registers
// allow two workgroups per CU either way).  A term row holds RP float4
// slices (8 in the split buffers, 16 otherwise) and thread tid always moves
// slice `tid % RP` of terms tid/RP + (NT/RP)j, so the LDS destination of a
// wave's DMA is contiguous (lane * 16 bytes), as the instruction requires.
// Lane (kk, ln): pair kk of the current MFMA k-step, 2 lines x QZL qz.

constexpr int kFoldUnits = 4;  // units (32 pairs) per FP64 fold of the FP32 MFMA sums
constexpr int kWStride = 34;   // float2 per term row of W (32 lines + pad)
constexpr int kNPT = kMaxChunkTerms;   // 72 terms per chunk at most
constexpr int kParts = 16;     // float4 slices per term row of a raw buffer holding all three axes

typedef __attribute__((address_space(3))) void lds_void_t;

template <typename T>
__device__ __forceinline__ uint32_t lds_addr(T* p) { return (uint32_t)(uintptr_t)(lds_void_t*)p; }

// 16 bytes per lane from sbase + voff (sbase wave-uniform, voff per lane) to
// LDS at lds_byte + 16 * lane (lds_byte wave-uniform).  Issued as inline
// assembly so that the compiler does not treat every later LDS read as a
// possible alias of the in-flight copy (it would then wait for all outstanding
// vector-memory operations before each of them); completion is awaited
// explicitly by barrier_dma.
__device__ __forceinline__ void dma_b128(uint32_t voff, const void* sbase, uint32_t lds_byte) {
    const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_byte);
    // the base is wave-uniform; say so, so that it lives in scalar registers
    // also where it was loaded from memory (the batch kernel's descriptors)
    // (readfirstlane returns a signed int: each half is widened through
    // uint32_t, never sign-extended into the other half)
    const uint64_t b = (uint64_t)(uintptr_t)sbase;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    const uint64_t bu = ((uint64_t)hi << 32) | (uint64_t)lo;
    // s_nop 4: five wait states between a VALU write of the base or M0
    // (v_readfirstlane) and their read by the VMEM instruction, which the
    // compiler cannot see inside the asm; also covers the M0 write (one)
    asm volatile("s_nop 4\n\tglobal_load_lds_dwordx4 %0, %1" ::"v"(voff), "s"(bu), "{m0}"(m0) : "memory");
}

typedef int sint4 __attribute__((ext_vector_type(4)));

// One 16-byte entry of a wave-uniform table (the chunk table) read through
// the scalar cache into scalar registers.  A load the compiler would issue
// itself after the DMA asm (which clobbers memory) goes through vector
// memory, and its wait would also wait for the DMA in flight.  The wait for
// the result is in the same asm block; s_nop 4 covers a VALU-written base.
__device__ __forceinline__ int4 sload_int4(const int4* p) {
    const uint64_t b = (uint64_t)(uintptr_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    const uint64_t bu = ((uint64_t)hi << 32) | (uint64_t)lo;
    sint4 r;
    asm volatile("s_nop 4\n\ts_load_dwordx4 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(bu) : "memory");
    return make_int4(r.x, r.y, r.z, r.w);
}

// LDS-only barrier: prior LDS reads/writes of this wave complete, DMA may
// still be in flight.
__device__ __forceinline__ void barrier_lds() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
// Full barrier: this wave's DMA into LDS has landed as well.  The wait is the
// compiler's own s_waitcnt (vmcnt(0) lgkmcnt(0)), so it knows that every
// earlier vector-memory load is complete here.
__device__ __forceinline__ void barrier_dma() {
    __builtin_amdgcn_s_waitcnt(0x0070);
    asm volatile("s_barrier" ::: "memory");
}

// One tile of one evaluation (blk = split * tiles + tile, as the single-request
// launch numbers its workgroups).  Shared by the single-request kernel (one
// tile per workgroup) and the persistent batch kernel (tiles of several
// requests popped from a queue), so a tile's values do not depend on which
// of the two computed it.
template <int SB, int QZL, bool BF, int NW>
__device__ __forceinline__ void grid_tile(const GridDesc& d, int blk) {
    const float2* __restrict__ V = d.V;
    const int vstride = d.vstride, vrows = d.vrows;
    const int4* __restrict__ terms = d.terms;
    const int4* __restrict__ chunks = d.chunks;
    const ChunkSplit& sp = d.sp;
    const uint32_t* __restrict__ Tp = d.Tp;
    const int3 n = d.n, ntiles = d.ntiles;
    const int nx_eval = d.nx_eval, n_states = d.n_states;
    float2* __restrict__ f = d.f;
    float* __restrict__ f2 = d.f2;
    double2* __restrict__ partial = d.partial;
    const long long part_stride = d.part_stride;

    constexpr int NT = NW * 64;        // threads
    constexpr int ZH = NW / 4;         // waves per q_x line of the tile (q_z halves)
    constexpr int TZ = 4 * QZL * ZH;   // q_z values of the tile
    constexpr int ZPARTS = TZ / 2;     // float4 slices of a Z row
    constexpr int SLOTS = 2 * QZL;     // q values per lane
    constexpr int SW = 16 * SB;        // padded state count
    // V^x / V^y in a buffer of their own (one state block), or all slices of a
    // term in one row of the double-buffered raw buffer
    constexpr bool SXY = SB == 1;
    constexpr int RP = SXY ? 8 : kParts;      // float4 slices per term row of a raw buffer
    constexpr int ZOFF = SXY ? 0 : 6;         // first V^z slice of a row
    constexpr int TPW8 = 64 / RP;             // terms per wave per DMA pass
    constexpr int TPP = NT / RP;              // terms per DMA pass (RP slice-threads per term)
    constexpr int NJ = (kNPT + TPP - 1) / TPP;   // term groups per slice-thread
    static_assert(NW == 4 || NW == 8, "4 or 8 waves per workgroup");
    constexpr int TPW = kMaxUnitsPerChunk * kChunk * SW;   // Tp words per chunk at most
    static_assert(SXY ? (2 + 4 <= RP && ZPARTS <= RP) : (2 + 4 + ZPARTS <= RP), "slices per term");
    static_assert(QZL % 2 == 0, "q_z values per lane come in float4 pairs");
    static_assert(TPW / 4 <= 256, "Tp block per chunk fits one DMA per thread");
    // software prefetch of the next term's LDS slices (12 VGPRs): only where
    // the register budget has room for it (not next to the 128 VGPRs of FP64
    // fold totals that the FP32 path needs at QZL = 4)
    constexpr bool PF = BF || QZL <= 2;

    // raw slice buffers: V^z (split) or all slices (not split), double-buffered
    __shared__ __align__(16) float4 Z0[kNPT * RP];
    __shared__ __align__(16) float4 Z1[kNPT * RP];
    __shared__ __align__(16) float4 XY[SXY ? kNPT * RP : 1];
    // Tp words: FP32 bits, or (BF) hi | lo << 16 split-BF16 halves
    __shared__ __align__(16) uint32_t T0[TPW];
    __shared__ __align__(16) uint32_t T1[TPW];
    __shared__ __align__(16) float2 Wl[kNPT * kWStride];

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wxq = wave & 3;          // q_x line of the tile
    const int wzh = wave >> 2;         // q_z half of the tile (8 waves)
    const int lane = tid & 63;
    const int kk = lane >> 4;          // pair within an MFMA k-step
    const int ln = lane & 15;          // MFMA column (q) / A-row (state) index
    const int lpair = ln >> 2;         // lines 2*lpair, 2*lpair+1 of the wave
    const int zgrp = ln & 3;           // qz values zgrp*QZL .. zgrp*QZL+QZL-1

    // block = (split of the chunk list, tile); a split sums chunks [c_lo, c_hi)
    int b = blk;
    const int split = b / (ntiles.x * ntiles.y * ntiles.z);
    b -= split * (ntiles.x * ntiles.y * ntiles.z);
    const int c_lo = sp.lo[split], c_hi = sp.lo[split + 1];
    const int tz = b % ntiles.z;
    b /= ntiles.z;
    const int ty = b % ntiles.y;
    const int tx = b / ntiles.y;
    const int qx0 = tx * 4, qy0 = ty * 8, qz0 = tz * TZ;

    // ---- this thread's slices: axis and offset of its 16 bytes in a table
    // row.  Split: for the V^x / V^y buffer (spare slices re-read a valid V^y
    // slice) and for the V^z buffer; not split: one slice of a whole row.
    // Idle slices re-read a valid V^z slice.
    const int part = tid & (RP - 1);
    const int axis_xy = part < 2 ? 0 : 1;
    const int qoff_xy = part < 2 ? qx0 + 2 * part : qy0 + 2 * min(part - 2, 3);
    const int axis_z = SXY ? 2 : (part < 2 ? 0 : (part < 6 ? 1 : 2));
    const int qoff_z = SXY ? qz0 + 2 * min(part, ZPARTS - 1)
                           : (part < 6 ? qoff_xy : qz0 + 2 * min(part - 6, ZPARTS - 1));

    // row ids of the slices of chunk c (loaded one chunk ahead of the DMA)
    int rid_xy[NJ], rid_z[NJ];
    auto load_rows = [&](int c) {
        const int4 ch = sload_int4(chunks + c);   // (first unit, units, npp, first slot)
        const int nptl = ch.y * kChunk * ch.z;
        const int* tc = reinterpret_cast<const int*>(terms + ch.w);
        // lane indices recomputed here rather than kept live across the loop
        int t0 = threadIdx.x;
        asm volatile("" : "+v"(t0));
        const int p0 = SXY ? t0 >> 3 : t0 >> 4;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int* tr = tc + 4 * min(p0 + TPP * j, nptl - 1);
            if constexpr (SXY) rid_xy[j] = tr[axis_xy];
            rid_z[j] = tr[axis_z];
        }
    };
    // DMA of this thread's slices of a chunk into the raw buffer at rbase;
    // wave w of term group j covers terms TPP*j + TPW8*w .. + TPW8-1.  Row ids
    // are clamped to the table where they are used (after the barrier that
    // waits for their loads), so no DMA can leave the table whatever the slot
    // table holds
    auto dma_slices = [&](const int (&rid)[NJ], int qoff, uint32_t rbase) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            if (TPP * j + TPW8 * wave < kNPT) {
                const uint32_t r = min((uint32_t)rid[j], (uint32_t)(vrows - 1));
                dma_b128(8u * (__umul24(r, vstride) + qoff), V, rbase + (TPP * j + TPW8 * wave) * RP * 16);
            }
        }
    };
    // DMA of chunk c's V^x / V^y slices into XY (split buffers only)
    auto issue_dma_xy = [&]() {
        if constexpr (SXY) dma_slices(rid_xy, qoff_xy, lds_addr(XY));
    };
    // DMA of chunk c's V^z slices (or all its slices) into buffer zbase and
    // its Tp block into tbase
    auto issue_dma = [&](int c, uint32_t zbase, uint32_t tbase) {
        dma_slices(rid_z, qoff_z, zbase);
        const int4 ch = sload_int4(chunks + c);
        const int tpf4 = ch.y * (kChunk * SW / 4);   // float4 of Tp in this chunk
        if (64 * wave < tpf4 && lane < tpf4 - 64 * wave)
            dma_b128(16u * (64 * wave + lane), Tp + (size_t)ch.x * kChunk * SW, tbase + 1024 * wave);
    };

    floatx4 acc_r[SB][SLOTS], acc_i[SB][SLOTS];
    double tot_r[SB][SLOTS][4], tot_i[SB][SLOTS][4];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            acc_r[sb][s] = floatx4{0.f, 0.f, 0.f, 0.f};
            acc_i[sb][s] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < 4; ++i) tot_r[sb][s][i] = tot_i[sb][s][i] = 0.0;
        }
    // exact fold of the short FP32 MFMA block into FP64 totals (FP32 path)
    auto fold = [&]() {
#pragma unroll
        for (int sb = 0; sb < SB; ++sb)
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    tot_r[sb][s][i] += (double)acc_r[sb][s][i];
                    tot_i[sb][s][i] += (double)acc_i[sb][s][i];
                }
                acc_r[sb][s] = floatx4{0.f, 0.f, 0.f, 0.f};
                acc_i[sb][s] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
    };

    int units_done = 0;   // units contracted so far (fold cadence of the FP32 path)

    auto chunk_body = [&](int c, const float4* Z, const uint32_t* T, auto after_w) {
        const int4 ch = sload_int4(chunks + c);
        const int nu = ch.y;
        const int npp = ch.z;
        // W = Vx * Vy: item = (term, qx, pair of q_y lines).  The 16 items of
        // a term are 16 consecutive threads, so the LDS reads of a quarter
        // wave touch one term row (no two terms' rows, 64 dwords apart, meet
        // in a bank).  The thread index is re-read (not kept live across the
        // loop) to spare a register.
        int i0 = threadIdx.x;
        asm volatile("" : "+v"(i0));
        for (int i = i0; i < nu * kChunk * npp * 16; i += NT) {
            const int ptl = i >> 4, xq = (i >> 2) & 3, h = i & 3;
            const float4* xy = SXY ? XY : Z;   // this chunk's V^x / V^y
            const float2 vx = reinterpret_cast<const float2*>(xy + ptl * RP)[xq];
            const float4 y = xy[ptl * RP + 2 + h];
            reinterpret_cast<float4*>(Wl + ptl * kWStride + xq * 8)[h] =
                make_float4(vx.x * y.x - vx.y * y.y, vx.x * y.y + vx.y * y.x, vx.x * y.z - vx.y * y.w,
                            vx.x * y.w + vx.y * y.z);
        }
        barrier_lds();
        after_w();   // XY is free: the next chunk's V^x / V^y DMA
        // G of one component pair (index p in the chunk) for this lane's 2
        // lines x QZL q_z values, G = sum_t W_t(line) Vz_t(qz).  The first term
        // initialises G; in the prefetching variant the slices of term t+1 are
        // read from LDS while the FMAs of term t run.
        auto gen = [&](int p, float (&gr)[SLOTS], float (&gi)[SLOTS]) {
            // 24-bit index arithmetic: keeps the compiler from forming 64-bit
            // multiply-adds whose unused high half may name a register with a
            // load still in flight (which would make it wait for that load)
            const int pt = __umul24(p, npp);
            const float2* wp = Wl + (__umul24(pt, kWStride) + wxq * 8 + 2 * lpair);
            const float2* zp = reinterpret_cast<const float2*>(Z) +
                               (__umul24(pt, 2 * RP) + 2 * ZOFF + wzh * (4 * QZL) + zgrp * QZL);
            auto load = [&](int t, float4& w, float4 (&zz)[QZL / 2]) {
                w = *reinterpret_cast<const float4*>(wp + t * kWStride);
#pragma unroll
                for (int j = 0; j < QZL / 2; ++j) zz[j] = *reinterpret_cast<const float4*>(zp + t * (2 * RP) + 2 * j);
            };
            auto zval = [&](const float4 (&zz)[QZL / 2], int j) {
                return (j & 1) ? make_float2(zz[j >> 1].z, zz[j >> 1].w) : make_float2(zz[j >> 1].x, zz[j >> 1].y);
            };
            auto fma_term = [&](const float4& w, const float4 (&zz)[QZL / 2]) {
#pragma unroll
                for (int j = 0; j < QZL; ++j) {
                    const float2 z = zval(zz, j);
                    gr[j] = fmaf(w.x, z.x, gr[j]);
                    gr[j] = fmaf(-w.y, z.y, gr[j]);
                    gi[j] = fmaf(w.x, z.y, gi[j]);
                    gi[j] = fmaf(w.y, z.x, gi[j]);
                    gr[QZL + j] = fmaf(w.z, z.x, gr[QZL + j]);
                    gr[QZL + j] = fmaf(-w.w, z.y, gr[QZL + j]);
                    gi[QZL + j] = fmaf(w.z, z.y, gi[QZL + j]);
                    gi[QZL + j] = fmaf(w.w, z.x, gi[QZL + j]);
                }
            };
            float4 wa, za[QZL / 2], wb, zb[QZL / 2];
            load(0, wa, za);
            if (PF && npp > 1) load(1, wb, zb);
#pragma unroll
            for (int j = 0; j < QZL; ++j) {   // the first term initialises G
                const float2 z = zval(za, j);
                gr[j] = fmaf(-wa.y, z.y, wa.x * z.x);
                gi[j] = fmaf(wa.y, z.x, wa.x * z.y);
                gr[QZL + j] = fmaf(-wa.w, z.y, wa.z * z.x);
                gi[QZL + j] = fmaf(wa.w, z.x, wa.z * z.y);
            }
            if constexpr (PF) {
                // ping-pong register sets: (wb, zb) holds term t, (wa, za) term t+1
                int t = 1;
                for (; t + 1 < npp; t += 2) {
                    load(t + 1, wa, za);
                    fma_term(wb, zb);
                    load(min(t + 2, npp - 1), wb, zb);   // clamped: no conditional register set
                    fma_term(wa, za);
                }
                if (t < npp) fma_term(wb, zb);
            } else {
                for (int t = 1; t < npp; ++t) {
                    load(t, wa, za);
                    fma_term(wa, za);
                }
            }
        };
        for (int u = 0; u < nu; ++u) {
            // two MFMA k-steps of 4 pairs each; lane (kk, ln) handles pair 4*step + kk of the unit
            float gr[2][SLOTS], gi[2][SLOTS];
            uint32_t a_op[2][SB];
#pragma unroll
            for (int step = 0; step < kChunk / 4; ++step) {
                const int p = u * kChunk + step * 4 + kk;
#pragma unroll
                for (int sb = 0; sb < SB; ++sb) a_op[step][sb] = T[p * SW + sb * 16 + ln];
                gen(p, gr[step], gi[step]);
                if constexpr (!BF) {
                    // raised wave priority while the matrix instructions
                    // issue (four-wave variants; the eight-wave one measured
                    // slower with it)
                    if constexpr (NW == 4) __builtin_amdgcn_s_setprio(1);
#pragma unroll
                    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
                        for (int s = 0; s < SLOTS; ++s) {
                            const float a = __uint_as_float(a_op[step][sb]);
                            acc_r[sb][s] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, gr[step][s], acc_r[sb][s], 0, 0, 0);
                            acc_i[sb][s] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, gi[step][s], acc_i[sb][s], 0, 0, 0);
                        }
                    if constexpr (NW == 4) __builtin_amdgcn_s_setprio(0);
                }
            }
            ++units_done;
            if constexpr (BF) {
                // Split-BF16 contraction of this unit in one 16x16x32 MFMA per
                // output block.  A lane's eight k-items are its two k-steps
                // (pairs kk and 4 + kk of the unit) four times over:
                //   A = (Tp lo | 0 | Tp hi | Tp hi),  B = (G hi | G lo | G hi | G lo)
                // so the items give lo*hi, 0, hi*hi, hi*lo.  A and B map lane and
                // item to k alike, so this item order is a valid k order.  One
                // unit per MFMA, so no state is carried between units (pairing
                // units for a 16-pair group made the compiler copy the
                // accumulators on every unit).
                // The split and the matrix instructions run at raised wave
                // priority, so that a wave holding a unit's products is issued
                // ahead of a wave in its generator loop on the same SIMD.
                __builtin_amdgcn_s_setprio(1);
                uint32_t hr[SLOTS], lr[SLOTS], hi[SLOTS], li[SLOTS];
#pragma unroll
                for (int s = 0; s < SLOTS; ++s) {
                    split_bf16(gr[0][s], gr[1][s], hr[s], lr[s]);
                    split_bf16(gi[0][s], gi[1][s], hi[s], li[s]);
                }
#pragma unroll
                for (int sb = 0; sb < SB; ++sb) {
                    const uint32_t ah = (a_op[0][sb] & 0xffffu) | (a_op[1][sb] << 16);
                    const uint32_t al = (a_op[0][sb] >> 16) | (a_op[1][sb] & 0xffff0000u);
                    const bf16x8 A = bf16x8_of(al, 0u, ah, ah);
#pragma unroll
                    for (int s = 0; s < SLOTS; ++s) {
                        const bf16x8 Br = bf16x8_of(hr[s], lr[s], hr[s], lr[s]);
                        const bf16x8 Bi = bf16x8_of(hi[s], li[s], hi[s], li[s]);
                        acc_r[sb][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Br, acc_r[sb][s], 0, 0, 0);
                        acc_i[sb][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bi, acc_i[sb][s], 0, 0, 0);
                    }
                }
                __builtin_amdgcn_s_setprio(0);
            } else {
                if ((units_done & (kFoldUnits - 1)) == 0) fold();
            }
        }
    };

    if (c_hi > c_lo) {
        load_rows(c_lo);
        issue_dma_xy();
        issue_dma(c_lo, lds_addr(Z0), lds_addr(T0));
        if (c_lo + 1 < c_hi) load_rows(c_lo + 1);
    }
    // two chunks per iteration so each buffer is a distinct LDS object.  The
    // row ids held at the start of chunk c are chunk c+1's: its V^z / Tp DMA
    // goes out at once, its V^x / V^y DMA once chunk c's W phase has read XY,
    // and then the row ids of chunk c+2 are loaded
    for (int c = c_lo; c < c_hi; c += 2) {
        barrier_dma();                                  // chunk c landed in Z0/T0 (and XY); Z1, T1 and Wl are free
        if (c + 1 < c_hi) {
            issue_dma(c + 1, lds_addr(Z1), lds_addr(T1));
            if (!SXY && c + 2 < c_hi) load_rows(c + 2);
        }
        chunk_body(c, Z0, T0, [&]() {
            if (SXY && c + 1 < c_hi) {
                issue_dma_xy();
                if (c + 2 < c_hi) load_rows(c + 2);
            }
        });
        if (c + 1 >= c_hi) break;
        barrier_dma();                                  // chunk c+1 landed in Z1/T1 (and XY); Z0, T0 and Wl are free
        if (c + 2 < c_hi) {
            issue_dma(c + 2, lds_addr(Z0), lds_addr(T0));
            if (!SXY && c + 3 < c_hi) load_rows(c + 3);
        }
        chunk_body(c + 1, Z1, T1, [&]() {
            if (SXY && c + 2 < c_hi) {
                issue_dma_xy();
                if (c + 3 < c_hi) load_rows(c + 3);
            }
        });
    }
    if constexpr (!BF) {
        if (units_done & (kFoldUnits - 1)) fold();
    }

    // Epilogue, coalesced through LDS.  Lane (kk, ln) holds states
    // sb*16 + 4kk + i of its q values (lines 2*lpair + a, q_z zgrp*QZL + j).
    // One pass per (sb, i, a): every lane writes its QZL values to the wave's
    // own LDS region as 16 rows (kk, lpair) of 4*QZL q_z, then the wave reads
    // the rows back with consecutive lanes on consecutive q_z and stores them,
    // so every row of the output (fixed state, q_x, q_y) is written as one
    // contiguous run.  The staging reuses the W buffer and a V^z buffer (no
    // wave reads them after the barrier below, and no DMA is in flight).
    constexpr int RQ = 4 * QZL;          // q_z values of a row
    constexpr int RPI = 64 / RQ;         // rows per wave-wide read
    barrier_lds();
    const int qx = qx0 + wxq;
    const bool plane_ok = qx < nx_eval;
    // per wave: 16 rows x RQ values; f (float2) or partial (double2) in Wl
    // (split) or Z0, f2 (float) in Z0 (split) or Z1
    static_assert(SXY ? (NW * 16 * RQ * sizeof(double2) <= sizeof(Wl) && NW * 16 * RQ * sizeof(float) <= sizeof(Z0))
                      : (NW * 16 * RQ * sizeof(double2) <= sizeof(Z0) && NW * 16 * RQ * sizeof(float) <= sizeof(Z1)),
                  "epilogue staging fits");
    void* s_f = SXY ? (void*)Wl : (void*)Z0;
    double2* sp2 = reinterpret_cast<double2*>(s_f) + wave * 16 * RQ;
    float2* sf = reinterpret_cast<float2*>(s_f) + wave * 16 * RQ;
    float* sf2 = reinterpret_cast<float*>(SXY ? Z0 : Z1) + wave * 16 * RQ;
    const int wrow = kk * 4 + lpair;     // the row this lane's values belong to
#pragma unroll
    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
#pragma unroll
                for (int j = 0; j < QZL; ++j) {
                    const int sl = a * QZL + j;
                    const double vr = BF ? (double)acc_r[sb][sl][i] : tot_r[sb][sl][i];
                    const double vi = BF ? (double)acc_i[sb][sl][i] : tot_i[sb][sl][i];
                    const int e = wrow * RQ + zgrp * QZL + j;
                    if (partial) {
                        sp2[e] = make_double2(vr, vi);
                    } else {
                        sf[e] = make_float2((float)vr, (float)vi);
                        sf2[e] = (float)(vr * vr + vi * vi);
                    }
                }
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // this wave's rows are in LDS
#pragma unroll
                for (int r0 = 0; r0 < 16; r0 += RPI) {
                    const int row = r0 + lane / RQ, col = lane % RQ;
                    const int rk = row >> 2, rl = row & 3;
                    const int st = sb * 16 + 4 * rk + i;
                    const int qy = qy0 + 2 * rl + a;
                    const int qz = qz0 + wzh * RQ + col;
                    const int e = row * RQ + col;
                    if (plane_ok && st < n_states && qy < n.y && qz < n.z) {
                        const size_t o = (((size_t)st * n.x + qx) * n.y + qy) * n.z + qz;
                        if (partial) {   // split pair sum: FP64 partial, summed by reduce_kernel
                            partial[(size_t)split * part_stride + o] = sp2[e];
                        } else {
                            if (f) f[o] = sf[e];
                            if (f2) f2[o] = sf2[e];
                        }
                    }
                }
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // read before the next pass writes
            }
}

template <int SB, int QZL, int WPE, bool BF, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void grid_kernel(GridDesc d) {
    grid_tile<SB, QZL, BF, NW>(d, blockIdx.x);
}

// Persistent batch kernel: every workgroup pops (request, tile) items from a
// device queue (items[i] = (descriptor index, tile of that request's launch))
// through an atomic counter until the queue is exhausted, so the tiles of
// several requests share one launch.  Every workgroup leaves the loop once
// the counter passes n_items; the counter must be 0 at launch.
template <int SB, int QZL, int WPE, bool BF, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void grid_batch_kernel(
    const GridDesc* __restrict__ descs, const int2* __restrict__ items, int n_items, int* __restrict__ counter) {
    __shared__ int s_item;
    for (;;) {
        __syncthreads();   // the previous tile's LDS use (epilogue staging) is over
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= n_items) break;
        const int2 w = items[it];
        grid_tile<SB, QZL, BF, NW>(descs[w.x], w.y);
    }
}

// Zeroes the batch queue counters (a kernel rather than a memset, so a
// captured graph replays it faithfully).
__global__ void zero_counters_kernel(int* __restrict__ c, int n) {
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

// ---------------------------------------------------------------- split reduction
//
// Sum of the FP64 partial results of the chunk-list splits (fixed order) for
// the evaluated planes ix < nx_eval, then f and |f|^2 as from the grid kernel.

__global__ void reduce_kernel(const double2* __restrict__ part, int n_split, long long stride, int3 n,
                              int nx_eval, int n_states, float2* __restrict__ f, float* __restrict__ f2) {
    const long long per_s = (long long)nx_eval * n.y * n.z;
    const long long tot = per_s * n_states;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < tot;
         i += (long long)gridDim.x * blockDim.x) {
        const int s = (int)(i / per_s);
        long long r = i - (long long)s * per_s;
        const int iz = (int)(r % n.z);
        r /= n.z;
        const int iy = (int)(r % n.y);
        const int ix = (int)(r / n.y);
        const size_t o = (((size_t)s * n.x + ix) * n.y + iy) * n.z + iz;
        double re = 0.0, im = 0.0;
        for (int j = 0; j < n_split; ++j) {
            const double2 v = part[(size_t)j * stride + o];
            re += v.x;
            im += v.y;
        }
        if (f) f[o] = make_float2((float)re, (float)im);
        if (f2) f2[o] = (float)(re * re + im * im);
    }
}

// ---------------------------------------------------------------- mirror kernel
//
// For a real transition density the form factor obeys f(-q) = f(q)* (the
// integrand's phase e^{iq.r} is conjugated by q -> -q, everything else is
// real).  On a grid symmetric about q = 0 (q_min = -q_max on every axis) the
// point with indices (nx-1-ix, ny-1-iy, nz-1-iz) is -q of (ix, iy, iz), so
// the grid kernel evaluates the planes ix < nx_eval = ceil(nx/2) and this
// kernel writes the others as conjugates: f[s][ix][iy][iz] =
// conj(f[s][nx-1-ix][ny-1-iy][nz-1-iz]), |f|^2 copied.

__global__ void mirror_kernel(int3 n, int nx_eval, int n_states, float2* __restrict__ f, float* __restrict__ f2) {
    const long long per_s = (long long)(n.x - nx_eval) * n.y * n.z;
    const long long tot = per_s * n_states;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < tot;
         i += (long long)gridDim.x * blockDim.x) {
        const int s = (int)(i / per_s);
        long long r = i - (long long)s * per_s;
        const int iz = (int)(r % n.z);
        r /= n.z;
        const int iy = (int)(r % n.y);
        const int ix = nx_eval + (int)(r / n.y);
        const size_t o = (((size_t)s * n.x + ix) * n.y + iy) * n.z + iz;
        const size_t m = (((size_t)s * n.x + (n.x - 1 - ix)) * n.y + (n.y - 1 - iy)) * n.z + (n.z - 1 - iz);
        if (f) {
            const float2 v = f[m];
            f[o] = make_float2(v.x, -v.y);
        }
        if (f2) f2[o] = f2[m];
    }
}

// ---------------------------------------------------------------- points kernel

template <int SB>
__global__ __launch_bounds__(64) void points_kernel(
    const VRowDev* __restrict__ rows, const int4* __restrict__ terms,
    const int* __restrict__ chunk_off, const int* __restrict__ chunk_npp, int n_units,
    const float* __restrict__ Tp, const double* __restrict__ qpts, int nq, int n_states,
    float2* __restrict__ f, float* __restrict__ f2) {
    constexpr int SW = 16 * SB;
    const int iq = blockIdx.x * blockDim.x + threadIdx.x;
    if (iq >= nq) return;
    const double qx = qpts[3 * iq], qy = qpts[3 * iq + 1], qz = qpts[3 * iq + 2];
    // FP32 sums over the pairs of kPointFoldUnits units, folded into FP64
    // totals: the same accumulation as the grid kernel's FP32 path, which
    // bounds the rounding error of the long, cancelling pair sum
    float br[SW], bi[SW];
    double tr_[SW], ti[SW];
    for (int s = 0; s < SW; ++s) {
        br[s] = bi[s] = 0.f;
        tr_[s] = ti[s] = 0.0;
    }
    for (int c = 0; c < n_units; ++c) {
        const int npp = chunk_npp[c];
        const int4* tc = terms + chunk_off[c];
        for (int pair = 0; pair < kChunk; ++pair) {
            float gr = 0.f, gi = 0.f;
            for (int t = 0; t < npp; ++t) {
                const int4 tr = tc[pair * npp + t];
                if (!tr.w) continue;
                const float2 vx = eval_row(rows[tr.x], qx);
                const float2 vy = eval_row(rows[tr.y], qy);
                const float2 vz = eval_row(rows[tr.z], qz);
                const float wr = vx.x * vy.x - vx.y * vy.y, wi = vx.x * vy.y + vx.y * vy.x;
                gr = fmaf(wr, vz.x, fmaf(-wi, vz.y, gr));
                gi = fmaf(wr, vz.y, fmaf(wi, vz.x, gi));
            }
            const float* tp = Tp + (size_t)(c * kChunk + pair) * SW;
            for (int s = 0; s < n_states; ++s) {
                br[s] = fmaf(tp[s], gr, br[s]);
                bi[s] = fmaf(tp[s], gi, bi[s]);
            }
        }
        if ((c + 1) % kPointFoldUnits == 0 || c + 1 == n_units)
            for (int s = 0; s < SW; ++s) {
                tr_[s] += (double)br[s];
                ti[s] += (double)bi[s];
                br[s] = bi[s] = 0.f;
            }
    }
    for (int s = 0; s < n_states; ++s) {
        const double vr = tr_[s], vi = ti[s];
        const size_t o = (size_t)s * nq + iq;
        if (f) f[o] = make_float2((float)vr, (float)vi);
        if (f2) f2[o] = (float)(vr * vr + vi * vi);
    }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_vtable(const VRowDev* rows, int nrows, int vstride, const int n[3],
                         const double qmin[3], const double dq[3], float2* V, hipStream_t st) {
    const long long tot = (long long)nrows * vstride;
    int blocks = (int)((tot + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(vtable_kernel, dim3(blocks), dim3(256), 0, st, rows, nrows, vstride,
                       make_int3(n[0], n[1], n[2]), make_double3(qmin[0], qmin[1], qmin[2]),
                       make_double3(dq[0], dq[1], dq[2]), V);
    return hipGetLastError();
}

// Kernel variant of an evaluation: class = (state blocks - 1) + 2 * precision.
//   4 q_z per lane (8 q values) except for the FP32 contraction of 17..32
//   states (2 q_z per lane, 8 waves per tile), whose accumulators and FP64
//   fold totals would not fit 2 waves per SIMD otherwise.
// Every variant's tile covers 16 q_z values: 4 per lane on one wave per q_x
// line, or 2 per lane on two waves per line.  Workgroups resident per CU:
// three of 4 waves for split-BF16 with <= 16 states (156-160 VGPRs, 50 KB of
// LDS), one of 8 for FP32 with 17..32 states, two of 4 otherwise (their
// registers allow 2 waves per SIMD).
static int tile_qz(int, int) { return 16; }
int grid_wg_per_cu(int state_blocks, int precision) {
    if (state_blocks == 2 && precision == 0) return 1;
    return state_blocks == 1 && precision == 1 ? 3 : 2;
}
int grid_class(int state_blocks, int precision) { return (state_blocks - 1) + 2 * precision; }
static int class_waves(int cls) { return cls == 1 ? 8 : 4; }

long long grid_tiles(int state_blocks, int precision, const int n[3], int nx_eval) {
    const int tz = tile_qz(state_blocks, precision);
    return (long long)((nx_eval + 3) / 4) * ((n[1] + 7) / 8) * ((n[2] + tz - 1) / tz);
}

// Row stride of the 1D tables: every tile may read up to 16 values past the
// last grid point of an axis (zero padding written by vtable_kernel).
int vtable_stride(const int n[3]) {
    int m = n[0] > n[1] ? n[0] : n[1];
    m = m > n[2] ? m : n[2];
    return ((m + 15) / 16) * 16 + 16;
}

hipError_t grid_desc(int state_blocks, int precision, const float2* V, int vstride, int vrows, const int4* terms,
                     const int4* chunks, const ChunkSplit& sp, const float* Tp, const uint32_t* tp_bf,
                     const int n[3], int nx_eval, int n_states, float2* f, float* f2, double2* part, GridDesc* d,
                     long long* blocks) {
    if (precision != 0 && precision != 1) return hipErrorInvalidValue;
    if (state_blocks != 1 && state_blocks != 2) return hipErrorInvalidValue;
    if (vstride < vtable_stride(n) || vrows < 1) return hipErrorInvalidValue;
    if (nx_eval < 1 || nx_eval > n[0]) return hipErrorInvalidValue;
    if (sp.n < 1 || sp.n > kMaxSplit || sp.lo[0] != 0) return hipErrorInvalidValue;
    for (int j = 0; j < sp.n; ++j)
        if (sp.lo[j + 1] < sp.lo[j]) return hipErrorInvalidValue;
    if (sp.n > 1 && !part) return hipErrorInvalidValue;
    const int tz = tile_qz(state_blocks, precision);
    d->V = V;
    d->vstride = vstride;
    d->vrows = vrows;
    d->terms = terms;
    d->chunks = chunks;
    d->sp = sp;
    d->Tp = precision == 1 ? tp_bf : reinterpret_cast<const uint32_t*>(Tp);
    d->n = make_int3(n[0], n[1], n[2]);
    d->ntiles = make_int3((nx_eval + 3) / 4, (n[1] + 7) / 8, (n[2] + tz - 1) / tz);
    d->nx_eval = nx_eval;
    d->n_states = n_states;
    d->f = f;
    d->f2 = f2;
    d->partial = sp.n > 1 ? part : nullptr;
    d->part_stride = (long long)n_states * n[0] * n[1] * n[2];
    *blocks = (long long)d->ntiles.x * d->ntiles.y * d->ntiles.z * sp.n;
    return hipSuccess;
}

hipError_t launch_grid_desc(int cls, const GridDesc& d, long long blocks, hipStream_t st) {
    const dim3 grid((unsigned)blocks);
    switch (cls) {
        case 0: hipLaunchKernelGGL((grid_kernel<1, 4, 2, false, 4>), grid, dim3(256), 0, st, d); break;
        case 1: hipLaunchKernelGGL((grid_kernel<2, 2, 2, false, 8>), grid, dim3(512), 0, st, d); break;
        case 2: hipLaunchKernelGGL((grid_kernel<1, 4, 3, true, 4>), grid, dim3(256), 0, st, d); break;
        case 3: hipLaunchKernelGGL((grid_kernel<2, 4, 2, true, 4>), grid, dim3(256), 0, st, d); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Persistent launch over a queue of (descriptor, tile) items of class cls:
// `wgs` workgroups (the device's resident capacity), each looping until the
// queue is exhausted.  *counter must be 0 when the launch starts.
hipError_t launch_grid_batch(int cls, const GridDesc* descs, const int2* items, int n_items, int* counter, int wgs,
                             hipStream_t st) {
    if (n_items < 1 || wgs < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)wgs), block(class_waves(cls) * 64);
    switch (cls) {
        case 0: hipLaunchKernelGGL((grid_batch_kernel<1, 4, 2, false, 4>), grid, block, 0, st, descs, items, n_items, counter); break;
        case 1: hipLaunchKernelGGL((grid_batch_kernel<2, 2, 2, false, 8>), grid, block, 0, st, descs, items, n_items, counter); break;
        case 2: hipLaunchKernelGGL((grid_batch_kernel<1, 4, 3, true, 4>), grid, block, 0, st, descs, items, n_items, counter); break;
        case 3: hipLaunchKernelGGL((grid_batch_kernel<2, 4, 2, true, 4>), grid, block, 0, st, descs, items, n_items, counter); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_zero_counters(int* c, int n, hipStream_t st) {
    if (n < 1 || n > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(256), 0, st, c, n);
    return hipGetLastError();
}

hipError_t launch_grid(int state_blocks, int precision, const float2* V, int vstride, int vrows,
                       const int4* terms, const int4* chunks, const ChunkSplit& sp, const float* Tp,
                       const uint32_t* tp_bf, const int n[3], int nx_eval, int n_states, float2* f, float* f2,
                       double2* part, hipStream_t st) {
    GridDesc d;
    long long blocks = 0;
    const hipError_t e = grid_desc(state_blocks, precision, V, vstride, vrows, terms, chunks, sp, Tp, tp_bf, n,
                                   nx_eval, n_states, f, f2, part, &d, &blocks);
    if (e != hipSuccess) return e;
    return launch_grid_desc(grid_class(state_blocks, precision), d, blocks, st);
}

hipError_t launch_reduce(const double2* part, int n_split, const int n[3], int nx_eval, int n_states, float2* f,
                         float* f2, hipStream_t st) {
    if (n_split < 1 || nx_eval < 1 || nx_eval > n[0]) return hipErrorInvalidValue;
    const long long tot = (long long)nx_eval * n[1] * n[2] * n_states;
    int blocks = (int)((tot + 255) / 256);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(reduce_kernel, dim3(blocks), dim3(256), 0, st, part, n_split,
                       (long long)n_states * n[0] * n[1] * n[2], make_int3(n[0], n[1], n[2]), nx_eval, n_states, f,
                       f2);
    return hipGetLastError();
}

hipError_t launch_mirror(const int n[3], int nx_eval, int n_states, float2* f, float* f2, hipStream_t st) {
    // planes ix >= nx_eval mirror planes nx-1-ix < nx - nx_eval <= nx_eval (computed)
    if (nx_eval < (n[0] + 1) / 2 || nx_eval > n[0]) return hipErrorInvalidValue;
    if (nx_eval == n[0]) return hipSuccess;
    const long long tot = (long long)(n[0] - nx_eval) * n[1] * n[2] * n_states;
    int blocks = (int)((tot + 255) / 256);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(mirror_kernel, dim3(blocks), dim3(256), 0, st, make_int3(n[0], n[1], n[2]), nx_eval,
                       n_states, f, f2);
    return hipGetLastError();
}

hipError_t launch_points(int state_blocks, const VRowDev* rows, const int4* terms, const int* coff,
                         const int* cnpp, int n_units, const float* Tp, const double* q, int nq,
                         int n_states, float2* f, float* f2, hipStream_t st) {
    const int blocks = (nq + 63) / 64;
    if (state_blocks == 1)
        hipLaunchKernelGGL((points_kernel<1>), dim3(blocks), dim3(64), 0, st, rows, terms, coff, cnpp,
                           n_units, Tp, q, nq, n_states, f, f2);
    else
        hipLaunchKernelGGL((points_kernel<2>), dim3(blocks), dim3(64), 0, st, rows, terms, coff, cnpp,
                           n_units, Tp, q, nq, n_states, f, f2);
    return hipGetLastError();
}

}  // namespace scff
