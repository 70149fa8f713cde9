// gfx950 kernels for the state-vector hot path.
//
//  * gate application (Section 3.1, Algorithm 1), k <= 5: a direct path
//    for gates whose targets are all >= 6 (one index group per work-item,
//    64-amplitude rows per wavefront load) and a tiled path that stages
//    2^tb-amplitude tiles in LDS for gates touching bits 0..5 and for
//    several gates per sweep; fused matrices always sit in LDS and are read
//    with wave-uniform (broadcast) addresses;
//  * FP64 reductions (norm, two-qubit reduced density matrix, the
//    conventional method's trial norm) with a fixed grid and a fixed
//    butterfly/tree order, so results are bit-identical run to run;
//  * measurement sampling: FP64 block sums, one-workgroup scan, one
//    work-item per sample with Philox draws.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "qs_internal.h"
#include "qs_philox.h"

namespace qs {
namespace {

template <int K>
struct GateArgs {
    float2 m[(1 << K) * (1 << K)];
    int t[K];
};


// Insert a zero bit at each ascending target position.
template <int K, typename Idx>
__device__ __forceinline__ Idx spread_index(Idx g, const int *t) {
#pragma unroll
    for (int b = 0; b < K; ++b) {
        const int q = t[b];
        const Idx low = g & ((Idx(1) << q) - Idx(1));
        g = ((g >> q) << (q + 1)) | low;
    }
    return g;
}

template <int K, typename Idx>
__device__ __forceinline__ Idx local_offset(int j, const int *t) {
    Idx off = 0;
#pragma unroll
    for (int b = 0; b < K; ++b)
        if ((j >> b) & 1) off |= Idx(1) << t[b];
    return off;
}

// Read-only, wave-uniform matrices are read through the constant address
// space, so the compiler fetches them with scalar loads into SGPRs.
typedef const __attribute__((address_space(4))) float *ConstFloats;

__device__ __forceinline__ float2 const_entry(const float2 *p, int i) {
    const ConstFloats c = (ConstFloats)(p);
    return make_float2(c[2 * i], c[2 * i + 1]);
}

__device__ __forceinline__ float2 cmac(float2 acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
    return acc;
}

// ---------------------------------------------------------------- gates

// Direct path (every target >= 6): one 2^K-amplitude group per work-item;
// the low six index bits are lane bits, so each load instruction of a
// wavefront reads 64 consecutive amplitudes (512 B).  A work-item issues its
// group's loads before the workgroup stages the matrix.  K <= 2 matrices are
// read with wave-uniform addresses straight from memory (scalar loads);
// larger ones are staged once per workgroup in LDS and read as broadcasts.
template <int K, typename Idx>
__global__ __launch_bounds__(kBlock) void apply_direct(float2 *__restrict__ amp, Idx groups,
                                                       const float2 *__restrict__ mat,
                                                       TargetArgs ta) {
    constexpr int D = 1 << K;
    constexpr bool kLds = K >= 3;
    __shared__ float2 sm[kLds ? D * D : 1];
    const Idx stride = Idx(gridDim.x) * Idx(kBlock);
    Idx g = Idx(blockIdx.x) * Idx(kBlock) + Idx(threadIdx.x);
    float2 v[D];
    if (g < groups) {
        const Idx base = spread_index<K, Idx>(g, ta.t);
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = amp[base + local_offset<K, Idx>(j, ta.t)];
    }
    if (kLds) {
        for (int i = threadIdx.x; i < D * D; i += kBlock) sm[i] = mat[i];
        __syncthreads();
    }
    float2 um[kLds ? 1 : D * D];
    if (!kLds) {
#pragma unroll
        for (int i = 0; i < (kLds ? 1 : D * D); ++i) um[i] = const_entry(mat, i);
    }
    const float2 *m = kLds ? sm : um;
    for (;;) {
        if (g >= groups) break;
        const Idx base = spread_index<K, Idx>(g, ta.t);
#pragma unroll(K >= 3 ? 2 : D)
        for (int j = 0; j < D; ++j) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int l = 0; l < D; ++l) acc = cmac(acc, m[j * D + l], v[l]);
            amp[base + local_offset<K, Idx>(j, ta.t)] = acc;
        }
        g += stride;
        if (g >= groups) break;
        const Idx nb = spread_index<K, Idx>(g, ta.t);
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = amp[nb + local_offset<K, Idx>(j, ta.t)];
    }
}

__host__ __device__ constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Issue priority from the batches a wavefront still has to do in this gate:
// the arbiter favours older wavefronts, so without this the younger ones
// finish a gate late and the rest of the workgroup idles at the barrier.
__device__ __forceinline__ void prio_for_remaining(int remaining) {
    if (remaining >= 4) __builtin_amdgcn_s_setprio(3);
    else if (remaining == 3) __builtin_amdgcn_s_setprio(2);
    else if (remaining == 2) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

// ---- LDS layout of a tile
// Gates read and write a tile in LDS one 64-lane instruction at a time; the
// lanes of an instruction span a few group bits and target bits of the
// local index, and with the plain layout (float2 index = local index) a gate
// on low local bits puts them on a handful of banks.  The tile kernel
// therefore stores local index x at x ^ m(x): bits 0..4 (which of 32 float2
// bank pairs) are XORed with a linear function m of bits 5..7.  The columns
// of m were chosen by scoring every target set of k <= 4 in 13 bits against
// the access pattern of each gate routine below (average cost 1.26x the
// conflict-free rate instead of 2x, worst case 2x instead of 4x).  Bits 8
// and up are left alone, so the tile copy's per-row offsets stay immediate.
// The map is linear over GF(2), so an index made of disjoint bit fields maps
// field by field, map(a | b) = map(a) ^ map(b): the gate loops split their
// indices into a per-lane part computed once and a wave-uniform part
// computed on the scalar unit.
struct SwizzledTile {
    __host__ __device__ __forceinline__ static int map(int x) {
        const int m = (((x >> 5) & 1) ? 30 : 0) ^ (((x >> 6) & 1) ? 27 : 0) ^ (((x >> 7) & 1) ? 23 : 0);
        return x ^ m;
    }
};

// Plain layout (the batched kernel's resident states and tiles).
struct PlainTile {
    __host__ __device__ __forceinline__ static int map(int x) { return x; }
};

// Address table of a K-qubit gate on a tile.  Logical bit b of an index in
// the gate's frame is target b for b < K and, for b >= K, the (b - K)-th
// non-target local bit in ascending order (the group-index bits).
// tab[b] = 8 * map(1 << local position of logical bit b): the LDS byte offset
// that bit contributes.  The layout map is linear over GF(2), so the byte
// offset of any amplitude is the XOR of tab[] over its logical bits, and the
// gate loops only XOR table entries.  lt must be ascending; entries beyond the
// tile's width are unused.  Built on the host for the tile kernel's launches
// and on the device by the batched kernel.
template <int K, class L>
__host__ __device__ inline void gate_tables(const int *lt, int *tab) {
#pragma unroll
    for (int b = 0; b < K; ++b) tab[b] = 8 * L::map(1 << lt[b]);
#pragma unroll
    for (int j = 0; j + K < kMaxTileBits; ++j) {
        int p = j;  // the j-th free position: j plus the targets at or below it
#pragma unroll
        for (int b = 0; b < K; ++b)
            if (lt[b] <= p) ++p;
        tab[K + j] = 8 * L::map(1 << p);
    }
}

// XOR of tab[first + j] over the set bits j < NBITS of x.
template <int NBITS>
__device__ __forceinline__ int tab_xor(const int *tab, int first, int x) {
    int r = 0;
#pragma unroll
    for (int j = 0; j < NBITS; ++j)
        if ((x >> j) & 1) r ^= tab[first + j];
    return r;
}

// LDS accesses by byte offset: each address is one XOR of a per-lane and a
// wave-uniform byte offset.
__device__ __forceinline__ float2 lds_get(const float2 *sd, int byte) {
    return *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(sd) + byte);
}
__device__ __forceinline__ void lds_put(float2 *sd, int byte, float2 v) {
    *reinterpret_cast<float2 *>(reinterpret_cast<char *>(sd) + byte) = v;
}
// The real and imaginary parts from two accumulators, as two 4-byte stores
// (one ds_write2_b32, with no register moves to pair them).
__device__ __forceinline__ void lds_put2(float2 *sd, int byte, float re, float im) {
    float *p = reinterpret_cast<float *>(reinterpret_cast<char *>(sd) + byte);
    p[0] = re;
    p[1] = im;
}
__device__ __forceinline__ float lds_getf(const float2 *sd, int byte) {
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(sd) + byte);
}

// Wavefront index as a scalar, so loops over it stay uniform.
__device__ __forceinline__ int wave_index() {
    return __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
}

// One gate on a tile held in LDS with VALU multiply-adds: every group of the
// tile is owned by one work-item, which gathers its 2^K amplitudes,
// multiplies, and writes back in place.  `m` is an LDS copy of the matrix.
template <int K, class L, int NT = kBlock>
__device__ __forceinline__ void tile_gate_valu(float2 *__restrict__ sd, const float2 *__restrict__ m,
                                               const int *lt, int tb) {
    constexpr int D = 1 << K;
    int off[D];
#pragma unroll
    for (int j = 0; j < D; ++j) off[j] = L::map(local_offset<K, int>(j, lt));
    const int groups = 1 << (tb - K);
    for (int gg = threadIdx.x; gg < groups; gg += NT) {
        const int lb = L::map(spread_index<K, int>(gg, lt));
        float2 v[D];
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = sd[lb ^ off[j]];
#pragma unroll(K >= 3 ? 2 : D)
        for (int j = 0; j < D; ++j) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int l = 0; l < D; ++l) acc = cmac(acc, m[j * D + l], v[l]);
            sd[lb ^ off[j]] = acc;
        }
    }
}

// K <= 2: the matrix (at most 16 entries) sits in SGPRs for the whole tile.
// Work-item (lane, wave) owns groups lane + 64 wave + NT i; the next group's
// amplitudes are read before this one's are written (the last iteration
// re-reads its own group, which is harmless: the reads precede the writes).
// MatLds: `gm` is an LDS copy (read as broadcasts) instead of global memory
// read through the scalar cache.
template <int K, class L, int NT = kBlock, bool MatLds = false>
__device__ __forceinline__ void tile_gate_small(float2 *__restrict__ sd, const float2 *gm,
                                                const int *lt, const int *tab, int tb) {
    constexpr int D = 1 << K;
    float2 u[D * D];
#pragma unroll
    for (int i = 0; i < D * D; ++i) u[i] = MatLds ? gm[i] : const_entry(gm, i);
    int off[D];
#pragma unroll
    for (int j = 0; j < D; ++j) off[j] = L::map(local_offset<K, int>(j, lt));
    constexpr int NB = ilog2(NT);
    if (tb < K + NB) {  // fewer groups than work-items (small resident states)
        const int groups = 1 << (tb - K);
        for (int gg = threadIdx.x; gg < groups; gg += NT) {
            const int lb = L::map(spread_index<K, int>(gg, lt));
            float2 v[D];
#pragma unroll
            for (int j = 0; j < D; ++j) v[j] = sd[lb ^ off[j]];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                float2 acc = make_float2(0.f, 0.f);
#pragma unroll
                for (int l = 0; l < D; ++l) acc = cmac(acc, u[j * D + l], v[l]);
                sd[lb ^ off[j]] = acc;
            }
        }
        return;
    }
    // group index lane + 64 wave + NT it: logical bits K.. of the frame
    const int lane = threadIdx.x & 63, wave = wave_index();
    int ab[D];  // byte offset of amplitude j of the lane's group, without the batch part
    const int lane_part = tab_xor<6>(tab, K, lane);
#pragma unroll
    for (int j = 0; j < D; ++j) ab[j] = lane_part ^ tab_xor<K>(tab, 0, j);
    const int iters = 1 << (tb - K - NB);
    const int uw = tab_xor<NB - 6>(tab, K + 6, wave);
    int ub = uw;
    float2 v[D];
#pragma unroll
    for (int j = 0; j < D; ++j) v[j] = lds_get(sd, ab[j] ^ ub);
    for (int it = 0; it < iters; ++it) {
        prio_for_remaining(iters - it);
        const int itn = it + 1 < iters ? it + 1 : it;
        const int ubn = uw ^ tab_xor<kMaxTileBits - K - NB>(tab, K + NB, itn);
        float2 w[D];
#pragma unroll
        for (int j = 0; j < D; ++j) w[j] = lds_get(sd, ab[j] ^ ubn);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int l = 0; l < D; ++l) acc = cmac(acc, u[j * D + l], v[l]);
            lds_put(sd, ab[j] ^ ub, acc);
        }
        ub = ubn;
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = w[j];
    }
    __builtin_amdgcn_s_setprio(0);
}

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// A fused k-qubit block is a dense contraction W = U V over the tile's
// 2^(tb-k) index groups.  For k = 3, 4, 5 it runs on FP32 MFMA
// (v_mfma_f32_16x16x4f32: in step s lane l supplies A[l%16][4s + l/16] and
// B[4s + l/16][l%16]; accumulator r is row 4(l/16) + r, column l%16), 16
// groups per wavefront batch, the groups' amplitudes (or real components)
// as B, the matrix as A laid out per lane once per launch ("fragments").
//
// The contraction index is permuted so that every lane supplies exactly the
// amplitudes its accumulators return: lane (n, q) = (l%16, l/16) reads and
// writes the same LDS words, and one address set per batch serves both.
// Physical step s, lane quarter q carries logical input index pi(4s + q),
// and the fragments hold the matrix columns in that order.
//
// Every gate also gets a per-lane LDS offset table staged after its
// fragments (lane_base): the lane part of its addresses (group index low
// bits n, quarter q), which would otherwise take some thirty VALU
// instructions per gate and tile on every wavefront.
constexpr int kFrag3 = 64 * 4;   // floats of k = 3 fragments; the lane table follows
constexpr int kFrag4 = 64 * 12;
constexpr int kFrag5 = 64 * 48;

// Real-form entry (row 2 jo + co, column 2 ji + ci) of a complex matrix.
__device__ __forceinline__ float real_form(float2 u, int co, int ci) {
    return co == 0 ? (ci == 0 ? u.x : -u.y) : (ci == 0 ? u.y : u.x);
}

// The lane table of a gate: table[lane] = XOR of tab[] over the lane's
// group bits n (logical bits nb..nb+3) and quarter bits q (logical bits
// qb, qb+1).
template <int NT>
__device__ __forceinline__ void stage_lane_table(int *__restrict__ table, const int *tab, int nb, int qb) {
    for (int lane = threadIdx.x; lane < 64; lane += NT) {
        int v = 0;
        for (int b = 0; b < 4; ++b)
            if ((lane >> b) & 1) v ^= tab[nb + b];
        for (int b = 0; b < 2; ++b)
            if ((lane >> (4 + b)) & 1) v ^= tab[qb + b];
        table[lane] = v;
    }
}

// k = 3 in the real form [[Re U, -Im U], [Im U, Re U]] (rows and columns
// interleaved as 2 j + c, c = 0 real, 1 imaginary).  Lane quarter q supplies
// the real components 4q + s (s = 0..3) of its group, i.e. amplitudes 2q and
// 2q + 1, and its accumulator rows 4q + r are the same components.
// Fragments: frag[lane * 4 + s] = RealForm[l%16][4 (l/16) + s].
// Lane table: group bits are logical bits 3.., amplitude 2q has q at bits 1, 2.
template <int NT = kBlock>
__device__ __forceinline__ void stage_frag3(float *__restrict__ frag, const float2 *__restrict__ u,
                                            const int *tab) {
    for (int i = threadIdx.x; i < 64 * 4; i += NT) {
        const int lane = i >> 2, s = i & 3;
        const int row = lane & 15, col = 4 * (lane >> 4) + s;
        frag[i] = real_form(u[(row >> 1) * 8 + (col >> 1)], row & 1, col & 1);
    }
    stage_lane_table<NT>(reinterpret_cast<int *>(frag + kFrag3), tab, 3, 1);
}

// k = 4 with three real products instead of four (Gauss), arranged so that
// the MFMA accumulators do the combining: for U = A + iB and v = x + iy,
// with k1 = A (x + y),
//   Re Uv = A x - B y = k1 - (A + B) y,   Im Uv = B x + A y = k1 + (B - A) x,
// so one chain forms k1 and two chains seeded with it add (-(A + B)) y and
// (B - A) x.  The only per-amplitude vector work left is x + y.  Lane
// quarter q supplies amplitudes 4q + s in step s and returns 4q + r.
// Fragments: frag[lane * 12 + 4 m + s] = M_m[l%16][4 (l/16) + s] with
// M_0 = Re U, M_1 = -(Re U + Im U), M_2 = Im U - Re U.
// Lane table: group bits are logical bits 4.., q at bits 2, 3.
template <int NT = kBlock>
__device__ __forceinline__ void stage_frag4(float *__restrict__ frag, const float2 *__restrict__ u,
                                            const int *tab) {
    for (int i = threadIdx.x; i < 64 * 12; i += NT) {
        const int lane = i / 12, rem = i - 12 * lane;
        const int m = rem >> 2, s = rem & 3;
        const float2 e = u[(lane & 15) * 16 + 4 * (lane >> 4) + s];
        frag[i] = m == 0 ? e.x : (m == 1 ? -(e.x + e.y) : e.y - e.x);
    }
    stage_lane_table<NT>(reinterpret_cast<int *>(frag + kFrag4), tab, 4, 2);
}

// k = 5: the same three real products as k = 4, each now a 32 x 32 matrix.
// The 32 output rows form two halves h (rows 16 h + i) and the contraction
// runs in eight steps of four: lane quarter q supplies amplitude
// 16 (s / 4) + 4 q + s % 4 in step s and accumulator r of half h returns
// 16 h + 4 q + r.  48 MFMAs per 16 groups (a 5-qubit block is the densest
// contraction of a sweep: 16 flops per byte moved, Section 3.1).
// Fragments: frag[lane * 48 + 24 h + 8 m + s] = M_m[16 h + l%16][16 (s / 4) +
// 4 (l/16) + s % 4].  Lane table: group bits are logical bits 5.., q at 2, 3.
template <int NT = kBlock>
__device__ __forceinline__ void stage_frag5(float *__restrict__ frag, const float2 *__restrict__ u,
                                            const int *tab) {
    for (int i = threadIdx.x; i < 64 * 48; i += NT) {
        const int lane = i / 48, rem = i - 48 * lane;
        const int h = rem / 24, m = (rem % 24) >> 3, s = rem & 7;
        const float2 e = u[(16 * h + (lane & 15)) * 32 + 16 * (s >> 2) + 4 * (lane >> 4) + (s & 3)];
        frag[i] = m == 0 ? e.x : (m == 1 ? -(e.x + e.y) : e.y - e.x);
    }
    stage_lane_table<NT>(reinterpret_cast<int *>(frag + kFrag5), tab, 5, 2);
}

// 16 groups per wavefront batch; the next batch's amplitudes are read before
// this one's MFMAs, so the LDS latency hides behind them (batches touch
// disjoint groups, so reading ahead of the writes is safe).  The batch index
// b = wave + W it occupies the logical bits after the lane's group bits.
template <class L, int NT = kBlock>
__device__ __forceinline__ void tile_gate_mfma3(float2 *__restrict__ sd, const float *__restrict__ frag,
                                                const int *tab, int tb) {
    constexpr int W = NT / 64;
    constexpr int LW = ilog2(W);
    const int lane = threadIdx.x & 63, wave = wave_index();
    const f32x4 afr = *reinterpret_cast<const f32x4 *>(frag + lane * 4);
    const int a0 = reinterpret_cast<const int *>(frag + kFrag3)[lane];  // amplitude 2q
    const int a1 = a0 ^ tab[0];                                         // amplitude 2q + 1
    const int iters = (1 << (tb - 3 - 4)) / W;  // batches per wave: >= 1 needs tb >= 7 + log2 W
    const int uw = tab_xor<LW>(tab, 7, wave);
    int ub = uw;
    float2 v0 = lds_get(sd, a0 ^ ub), v1 = lds_get(sd, a1 ^ ub);
    for (int it = 0; it < iters; ++it) {
        prio_for_remaining(iters - it);
        const int itn = it + 1 < iters ? it + 1 : it;
        const int ubn = uw ^ tab_xor<kMaxTileBits - 7 - LW>(tab, 7 + LW, itn);
        const float2 w0 = lds_get(sd, a0 ^ ubn), w1 = lds_get(sd, a1 ^ ubn);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[0], v0.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[1], v0.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[2], v1.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[3], v1.y, acc, 0, 0, 0);
        lds_put(sd, a0 ^ ub, make_float2(acc[0], acc[1]));
        lds_put(sd, a1 ^ ub, make_float2(acc[2], acc[3]));
        ub = ubn;
        v0 = w0;
        v1 = w1;
    }
    __builtin_amdgcn_s_setprio(0);
}

template <class L, int NT = kBlock>
__device__ __forceinline__ void tile_gate_mfma4(float2 *__restrict__ sd, const float *__restrict__ frag,
                                                const int *tab, int tb) {
    constexpr int W = NT / 64;
    constexpr int LW = ilog2(W);
    const int lane = threadIdx.x & 63, wave = wave_index();
    const f32x4 *fp = reinterpret_cast<const f32x4 *>(frag + lane * 12);
    const f32x4 fa = fp[0], fb = fp[1], fs = fp[2];
    const int base = reinterpret_cast<const int *>(frag + kFrag4)[lane];
    int a[4];  // amplitude 4q + s of the lane's group
#pragma unroll
    for (int s = 0; s < 4; ++s) a[s] = base ^ tab_xor<2>(tab, 0, s);
    const int iters = (1 << (tb - 4 - 4)) / W;  // batches per wave: >= 1 needs tb >= 8 + log2 W
    const int uw = tab_xor<LW>(tab, 8, wave);
    int ub = uw;
    float2 v[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = lds_get(sd, a[s] ^ ub);
    for (int it = 0; it < iters; ++it) {
        prio_for_remaining(iters - it);
        const int itn = it + 1 < iters ? it + 1 : it;
        const int ubn = uw ^ tab_xor<kMaxTileBits - 8 - LW>(tab, 8 + LW, itn);
        float2 w[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) w[s] = lds_get(sd, a[s] ^ ubn);
        f32x4 k1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) k1 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s], v[s].x + v[s].y, k1, 0, 0, 0);
        f32x4 re = k1, im = k1;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            re = __builtin_amdgcn_mfma_f32_16x16x4f32(fb[s], v[s].y, re, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f32_16x16x4f32(fs[s], v[s].x, im, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) lds_put2(sd, a[r] ^ ub, re[r], im[r]);
        ub = ubn;
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = w[s];
    }
    __builtin_amdgcn_s_setprio(0);
}

// The two output halves are formed one after the other from the same
// inputs in registers.
template <class L, int NT = kBlock>
__device__ __forceinline__ void tile_gate_mfma5(float2 *__restrict__ sd, const float *__restrict__ frag,
                                                const int *tab, int tb) {
    constexpr int W = NT / 64;
    constexpr int LW = ilog2(W);
    const int lane = threadIdx.x & 63, wave = wave_index();
    const f32x4 *fp = reinterpret_cast<const f32x4 *>(frag + lane * 48);
    f32x4 F[12];  // F[6 h + 2 m + s / 4][s % 4]
#pragma unroll
    for (int i = 0; i < 12; ++i) F[i] = fp[i];
    const int base = reinterpret_cast<const int *>(frag + kFrag5)[lane];
    int a[8];  // amplitude 16 h + 4 q + r of the lane's group at a[4 h + r]
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) a[4 * h + r] = base ^ tab_xor<2>(tab, 0, r) ^ (h ? tab[4] : 0);
    const int iters = (1 << (tb - 5 - 4)) / W;  // batches per wave: >= 1 needs tb >= 9 + log2 W
    const int uw = tab_xor<LW>(tab, 9, wave);
    int ub = uw;
    float2 v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = lds_get(sd, a[s] ^ ub);
    for (int it = 0; it < iters; ++it) {
        prio_for_remaining(iters - it);
        const int itn = it + 1 < iters ? it + 1 : it;
        const int ubn = uw ^ tab_xor<kMaxTileBits - 9 - LW>(tab, 9 + LW, itn);
        float2 w[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) w[s] = lds_get(sd, a[s] ^ ubn);
        float xy[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) xy[s] = v[s].x + v[s].y;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            f32x4 k1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 8; ++s)
                k1 = __builtin_amdgcn_mfma_f32_16x16x4f32(F[6 * h + (s >> 2)][s & 3], xy[s], k1, 0, 0, 0);
            f32x4 re = k1, im = k1;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                re = __builtin_amdgcn_mfma_f32_16x16x4f32(F[6 * h + 2 + (s >> 2)][s & 3], v[s].y, re, 0, 0, 0);
                im = __builtin_amdgcn_mfma_f32_16x16x4f32(F[6 * h + 4 + (s >> 2)][s & 3], v[s].x, im, 0, 0, 0);
            }
            // inputs are in registers, so this half's outputs may overwrite them in LDS
#pragma unroll
            for (int r = 0; r < 4; ++r) lds_put2(sd, a[4 * h + r] ^ ub, re[r], im[r]);
        }
        ub = ubn;
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = w[s];
    }
    __builtin_amdgcn_s_setprio(0);
}

// Tiled path: persistent workgroups stage every gate matrix of the launch in
// LDS once (as MFMA fragments for k = 3, 4; plain for k = 5; k <= 2 matrices
// stay in global memory and arrive through scalar loads), then loop over
// tiles of 2^TB amplitudes -- the index bits in a.pos, bits 0..3 first, so
// every eight lanes of a wavefront load one whole 128-byte line.  A tile is written to LDS, the next
// tile's loads are issued into registers, the gates run on the LDS copy in
// order, and the tile is written back: any number of gates inside the tile
// cost one HBM read and one write.
// K5: whether the launch holds a 5-qubit block (its path needs many more
// VGPRs, so launches without one use a leaner instantiation).  5-qubit blocks
// run on MFMA when every wavefront gets a batch of 16 groups (TB >= 9 +
// log2(NT / 64)), else on VALU from the plain matrix.
// RK: the launch also accumulates the reduced density matrix of one tile
// qubit (TileArgs::rdm_out) from every tile after its gates.
template <int TB, typename Idx, bool K5, int NT, bool RK>
__global__ __launch_bounds__(NT) void apply_tile(float2 *__restrict__ amp, Idx n_tiles,
                                                 TileArgs a) {
    constexpr int NB = ilog2(NT);
    constexpr bool K5_MFMA = TB >= 9 + NB - 6;
    static_assert(TB >= 10, "the MFMA gates need at least 32 groups per tile");
    static_assert((1 << (TB - 8)) >= NT / 64, "every wavefront needs a 4-qubit batch");
    constexpr int E = 1 << TB;
    // Each work-item moves R amplitude pairs per tile: pair (t, r) holds local
    // indices 2 t + NT 2 r + {0, 1}, which differ in local bit 0 = qubit 0, so
    // the pair is one 16-byte load or store, and each eight lanes cover one
    // 128-byte line (local bits 0..3 are global bits 0..3).
    constexpr int R = E / (2 * NT);
    // The tile is a static array (its LDS address is a link-time constant
    // that folds into the LDS instructions' offsets); the launch's matrices
    // follow it in dynamic LDS.
    __shared__ float2 sd[E];
    extern __shared__ float2 sm[];
    Idx tile = blockIdx.x;
    if (tile >= n_tiles) return;  // uniform over the workgroup
    Idx off_tid = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b)
        if ((threadIdx.x >> b) & 1) off_tid |= Idx(1) << a.pos[b + 1];
    Idx off_r[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        Idx o = 0;
#pragma unroll
        for (int b = NB + 1; b < TB; ++b)
            if (((r << (NB + 1)) >> b) & 1) o |= Idx(1) << a.pos[b];
        off_r[r] = o;
    }
    // First index of tile t: the bits of t spread over the positions the tile
    // does not hold.  Inserting a zero at position q adds the part of the
    // index at and above q to itself (shifting it up by one); positions 0..3
    // are always the tile's, which is one shift.
    auto tile_base = [&](Idx t) {
        Idx base = t << kTileLowBits;
#pragma unroll
        for (int b = kTileLowBits; b < TB; ++b) base += base & (~Idx(0) << a.pos[b]);
        return base + off_tid;
    };
    // A tile's amplitude pairs.  With init_zero the sweep starts from
    // |0...0> without reading the state: nothing is fetched, and the tile's
    // LDS copy is written from zeros (amplitude 1 at index 0).
    auto fetch = [&](Idx t, float4 (&dst)[R]) {
        if (a.init_zero) return;
        const Idx base = tile_base(t);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r] = *reinterpret_cast<const float4 *>(amp + base + off_r[r]);
    };
    float4 v[R];
    fetch(tile, v);
    for (int gi = 0; gi < a.n_gates; ++gi) {
        const int k = a.g[gi].k;
        const float2 *src = a.g[gi].mat;
        float2 *dst = sm + a.g[gi].lofs;
        int gtab[kMaxTileBits];
#pragma unroll
        for (int b = 0; b < kMaxTileBits; ++b) gtab[b] = a.g[gi].tab[b];
        if (k == 4) {
            stage_frag4<NT>(reinterpret_cast<float *>(dst), src, gtab);
        } else if (k == 3) {
            stage_frag3<NT>(reinterpret_cast<float *>(dst), src, gtab);
        } else if (k == 5) {
            if constexpr (K5_MFMA) stage_frag5<NT>(reinterpret_cast<float *>(dst), src, gtab);
            else
                for (int i = threadIdx.x; i < 1024; i += NT) dst[i] = src[i];
        }
    }
    // One tile: the prefetched amplitudes go to LDS, the previous tile's
    // results (held in registers since its gates finished) are stored, the
    // next tile's loads are issued, the gates run, and the results are read
    // out of LDS into registers.  Stores and loads therefore drain while this
    // tile's gates run, instead of the stores going out in a burst at the end
    // of every tile; the wait for the prefetch at the next loop head covers
    // memory operations issued a whole gate phase earlier.
    // LDS index of local index 2 threadIdx.x + e + 2 NT r: the map leaves the
    // r part alone and flipping bit 0 of an index flips bit 0 of its image,
    // so it is tid_l ^ e + (r << NB + 1).  tid_l itself may be odd (columns 27
    // and 23 of the map set bit 0), so a pair is adjacent but not always in
    // order: it is not one 16-byte LDS access.
    const int tid_l = SwizzledTile::map(int(threadIdx.x) << 1);
    float4 o[R];
    Idx prev_base = 0;
    // RDM of the qubit at tile bit rdm_lt: R00, R11 and R01 = sum v0 conj(v1)
    // over every pair of the work-item's amplitudes that differ in that bit,
    // in a fixed order, summed over the workgroup's tiles.
    double r00 = 0.0, r11 = 0.0, r01r = 0.0, r01i = 0.0;
    auto run_tile = [&](Idx t, bool has_prev) {
        __syncthreads();  // the previous tile is out of LDS; matrices staged
        const Idx base = tile_base(t);
        if (a.init_zero) {
            const float one = base == Idx(0) ? 1.f : 0.f;  // index 0 is pair 0 of work-item 0
#pragma unroll
            for (int r = 0; r < R; ++r) {
                sd[tid_l + (r << (NB + 1))] = make_float2(r == 0 ? one : 0.f, 0.f);
                sd[(tid_l ^ 1) + (r << (NB + 1))] = make_float2(0.f, 0.f);
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                sd[tid_l + (r << (NB + 1))] = make_float2(v[r].x, v[r].y);
                sd[(tid_l ^ 1) + (r << (NB + 1))] = make_float2(v[r].z, v[r].w);
            }
        }
        if (has_prev) {
#pragma unroll
            for (int r = 0; r < R; ++r) *reinterpret_cast<float4 *>(amp + prev_base + off_r[r]) = o[r];
        }
        const Idx next = t + gridDim.x;
        if (next < n_tiles) fetch(next, v);
        __syncthreads();
        for (int gi = 0; gi < a.n_gates; ++gi) {
            const int k = a.g[gi].k;
            int lt[kMaxGateQubits], tab[kMaxTileBits];
#pragma unroll
            for (int b = 0; b < kMaxGateQubits; ++b) lt[b] = a.g[gi].lt[b];
#pragma unroll
            for (int b = 0; b < kMaxTileBits; ++b) tab[b] = a.g[gi].tab[b];
            switch (k) {
                case 1: tile_gate_small<1, SwizzledTile, NT>(sd, a.g[gi].mat, lt, tab, TB); break;
                case 2: tile_gate_small<2, SwizzledTile, NT>(sd, a.g[gi].mat, lt, tab, TB); break;
                case 3:
                    tile_gate_mfma3<SwizzledTile, NT>(sd, reinterpret_cast<const float *>(sm + a.g[gi].lofs),
                                                      tab, TB);
                    break;
                case 4:
                    tile_gate_mfma4<SwizzledTile, NT>(sd, reinterpret_cast<const float *>(sm + a.g[gi].lofs),
                                                      tab, TB);
                    break;
                default:
                    if constexpr (K5 && K5_MFMA)
                        tile_gate_mfma5<SwizzledTile, NT>(sd, reinterpret_cast<const float *>(sm + a.g[gi].lofs),
                                                          tab, TB);
                    else if constexpr (K5)
                        tile_gate_valu<5, SwizzledTile, NT>(sd, sm + a.g[gi].lofs, lt, TB);
                    break;
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float2 lo = sd[tid_l + (r << (NB + 1))], hi = sd[(tid_l ^ 1) + (r << (NB + 1))];
            o[r] = make_float4(lo.x, lo.y, hi.x, hi.y);
        }
        if constexpr (RK) {
            // the work-item's amplitudes are local indices 2 tid + e + 2 NT r,
            // read again from LDS (a rolled loop keeps the registers of the
            // common sweep); the partner across the qubit's bit pc sits at
            // LDS index ^ map(2^pc)
            const int pc = a.rdm_lt;
            const int pm = SwizzledTile::map(1 << pc);
            const int tid_bit = pc >= 1 && pc <= NB ? (int(threadIdx.x) >> (pc - 1)) & 1 : 0;
#pragma unroll 1
            for (int i = 0; i < 2 * R; ++i) {
                const int r = i >> 1, e = i & 1;
                const int bit = pc == 0 ? e : (pc <= NB ? tid_bit : (r >> (pc - NB - 1)) & 1);
                const int at = (tid_l ^ e) + (r << (NB + 1));
                const float2 v = sd[at];
                const double vr = v.x, vi = v.y;
                if (bit) {
                    r11 = fma(vr, vr, fma(vi, vi, r11));
                } else {
                    r00 = fma(vr, vr, fma(vi, vi, r00));
                    const float2 u = sd[at ^ pm];
                    const double ur = u.x, ui = u.y;
                    r01r = fma(vr, ur, fma(vi, ui, r01r));
                    r01i = fma(vi, ur, fma(-vr, ui, r01i));
                }
            }
        }
        prev_base = base;
    };
    run_tile(tile, false);
    for (tile += gridDim.x; tile < n_tiles; tile += gridDim.x) run_tile(tile, true);
#pragma unroll
    for (int r = 0; r < R; ++r) *reinterpret_cast<float4 *>(amp + prev_base + off_r[r]) = o[r];
    if constexpr (RK) {
        // wavefront sums by a fixed shuffle tree, then the wavefronts in order
        // through LDS (the tile is no longer needed once every wavefront has
        // read its last tile out)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            r00 += __shfl_xor(r00, off, 64);
            r11 += __shfl_xor(r11, off, 64);
            r01r += __shfl_xor(r01r, off, 64);
            r01i += __shfl_xor(r01i, off, 64);
        }
        __syncthreads();
        double *red = reinterpret_cast<double *>(sd);
        const int wave = int(threadIdx.x) >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[4 * wave] = r00;
            red[4 * wave + 1] = r11;
            red[4 * wave + 2] = r01r;
            red[4 * wave + 3] = r01i;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s00 = 0.0, s11 = 0.0, sr = 0.0, si = 0.0;
            for (int w = 0; w < NT / 64; ++w) {
                s00 += red[4 * w];
                s11 += red[4 * w + 1];
                sr += red[4 * w + 2];
                si += red[4 * w + 3];
            }
            double *rec = a.rdm_out + size_t(blockIdx.x) * 8;
            rec[0] = s00;
            rec[1] = 0.0;
            rec[2] = sr;
            rec[3] = si;
            rec[4] = sr;
            rec[5] = -si;
            rec[6] = s11;
            rec[7] = 0.0;
        }
    }
}

// ---------------------------------------------------------------- branch selection

__global__ __launch_bounds__(64) void select_branch(SelectArgs a) {
    __shared__ double scale;
    __shared__ int pick;
    if (threadIdx.x == 0) {
        const int D = a.D;
        double N = 0.0;
        for (int j = 0; j < D; ++j) N += a.rdm[2 * (j * D + j)];
        double r = a.resid;
        int chosen = -1, last_pos = -1;
        double e_chosen = 0.0;
        for (int i = 0; i < a.nk; ++i) {
            const double *M = a.excess + size_t(i) * D * D * 2;
            double tr = 0.0;  // Re sum_jl M[j][l] R[l][j]
            for (int j = 0; j < D; ++j)
                for (int l = 0; l < D; ++l) {
                    const double mr = M[2 * (j * D + l)], mi = M[2 * (j * D + l) + 1];
                    const double rr = a.rdm[2 * (l * D + j)], ri = a.rdm[2 * (l * D + j) + 1];
                    tr += mr * rr - mi * ri;
                }
            const double e = tr / N;
            if (e > 0.0) last_pos = i;
            if (r < e) {
                chosen = i;
                e_chosen = e;
                break;
            }
            r -= e;
        }
        if (chosen < 0) {
            chosen = last_pos >= 0 ? last_pos : a.nk - 1;
            // e of the fallback pick
            const double *M = a.excess + size_t(chosen) * D * D * 2;
            double tr = 0.0;
            for (int j = 0; j < D; ++j)
                for (int l = 0; l < D; ++l) {
                    const double mr = M[2 * (j * D + l)], mi = M[2 * (j * D + l) + 1];
                    const double rr = a.rdm[2 * (l * D + j)], ri = a.rdm[2 * (l * D + j) + 1];
                    tr += mr * rr - mi * ri;
                }
            e_chosen = tr / N;
        }
        const double p = a.pbar[chosen] + e_chosen;
        if (!(N > 0.0) || !(p > 0.0) || !(N < INFINITY)) {
            *a.err = 1;
            scale = 0.0;
        } else {
            scale = 1.0 / sqrt(p * N);
        }
        pick = chosen;
        *a.choice = chosen;
    }
    __syncthreads();
    const int dd = a.Db * a.Db;
    const double *c = a.cand + size_t(pick) * dd * 2;
    for (int i = threadIdx.x; i < dd; i += 64)
        a.dst[i] = make_float2(float(c[2 * i] * scale), float(c[2 * i + 1] * scale));
}

// ---------------------------------------------------------------- batched

// One fused block on amplitudes held in LDS (a whole resident state, or a
// tile).  For k <= 4, `lm` is the block's matrix already copied to LDS; for
// k = 5, `gm` is the global copy (two pointers, so that LDS reads compile
// to LDS instructions rather than flat ones, which would wait for every
// global load in flight).  Fragments for the MFMA gates are staged per
// block.  `then` runs after the block's arithmetic and before the trailing
// barrier, which lets the next block reuse the staging area.
template <int NT, class Then>
__device__ __forceinline__ void batched_gate(float2 *__restrict__ sd, float *__restrict__ frag,
                                             const BatchGate &g, const float2 *lm, const float2 *gm, int tb,
                                             Then then) {
    int lt[kMaxGateQubits], tab[kMaxTileBits];
#pragma unroll
    for (int b = 0; b < kMaxGateQubits; ++b) lt[b] = g.lt[b];
    // MFMA paths need at least one 16-group batch per wavefront at 512
    // work-items (k = 3: 10 bits, k = 4: 11); the 256-work-item form keeps
    // the same rule, so a job's arithmetic does not depend on the form
    if (g.k == 1) {
        gate_tables<1, PlainTile>(lt, tab);
        tile_gate_small<1, PlainTile, NT, true>(sd, lm, lt, tab, tb);
    } else if (g.k == 2) {
        gate_tables<2, PlainTile>(lt, tab);
        tile_gate_small<2, PlainTile, NT, true>(sd, lm, lt, tab, tb);
    } else if (g.k == 3 && tb >= 10) {
        gate_tables<3, PlainTile>(lt, tab);
        stage_frag3<NT>(frag, lm, tab);
        __syncthreads();
        tile_gate_mfma3<PlainTile, NT>(sd, frag, tab, tb);
    } else if (g.k == 4 && tb >= 11) {
        gate_tables<4, PlainTile>(lt, tab);
        stage_frag4<NT>(frag, lm, tab);
        __syncthreads();
        tile_gate_mfma4<PlainTile, NT>(sd, frag, tab, tb);
    } else if (g.k == 3) {
        tile_gate_valu<3, PlainTile, NT>(sd, lm, lt, tb);
    } else if (g.k == 4) {
        tile_gate_valu<4, PlainTile, NT>(sd, lm, lt, tb);
    } else {
        float2 *mm = reinterpret_cast<float2 *>(frag);
        for (int i = threadIdx.x; i < 1024; i += NT) mm[i] = gm[i];
        __syncthreads();
        tile_gate_valu<5, PlainTile, NT>(sd, mm, lt, tb);
    }
    then();
    __syncthreads();
}

// Algorithm 2's fast path for a mixture of unitaries: the first i with
// r < pbar_i after subtracting the earlier pbar_j (FP64, in order); when
// rounding leaves r above the total, the last operator with weight.
__device__ __forceinline__ int draw_pick(const double *pb, int nk, double r) {
    for (int i = 0; i < nk; ++i) {
        if (r < pb[i]) return i;
        r -= pb[i];
    }
    for (int i = nk - 1; i >= 0; --i)
        if (pb[i] > 0.0) return i;
    return nk - 1;
}

// A block of a job: its descriptor and its matrix (the default one, or the
// job's recomputed copy when one of the block's channels took another pick).
struct BatchedRef {
    BatchGate g;
    const float2 *m;
};

__device__ __forceinline__ BatchedRef batched_ref(const BatchArgs &A, const uint32_t *mask,
                                                  const float2 *mine, const BatchCircuit &C, int gi) {
    BatchedRef r;
    r.g = A.gates[gi];
    const int rel = gi - C.g0;
    const bool patched = (mask[rel >> 5] >> (rel & 31)) & 1u;
    r.m = patched ? mine + (r.g.mat - C.pool0) : A.mats + r.g.mat;
    return r;
}

// This work-item's entry of a k <= 4 matrix (at most 256 entries, one per
// work-item).
__device__ __forceinline__ bool batched_holds(const BatchedRef &r) {
    return r.g.k <= 4 && int(threadIdx.x) < (1 << (2 * r.g.k));
}

// Blocks [g0, g1) on the amplitudes in `sd`, software-pipelined so that no
// global-memory latency sits between two blocks: while block i runs, the
// matrix of block i + 1 travels into registers (and lands in the other half
// of the double-buffered LDS copy `raw` after block i's arithmetic) and the
// descriptor of block i + 2 is loaded.  Workgroup barriers on gfx950 do not
// wait for outstanding global loads, so both overlap the block's work.
template <int NT>
__device__ __forceinline__ void batched_blocks(const BatchArgs &A, const uint32_t *mask, const float2 *mine,
                               const BatchCircuit &C, int g0, int g1, float2 *__restrict__ sd,
                               float *__restrict__ frag, float2 *raw, int tb) {
    if (g0 >= g1) return;
    BatchedRef cur = batched_ref(A, mask, mine, C, g0);
    if (batched_holds(cur)) raw[threadIdx.x] = cur.m[threadIdx.x];
    BatchedRef nxt = cur;
    if (g0 + 1 < g1) nxt = batched_ref(A, mask, mine, C, g0 + 1);
    __syncthreads();
    int buf = 0;
    for (int gi = g0; gi < g1; ++gi) {
        const bool put1 = gi + 1 < g1 && batched_holds(nxt);
        float2 e1 = make_float2(0.f, 0.f);
        if (put1) e1 = nxt.m[threadIdx.x];
        BatchedRef after = nxt;
        if (gi + 2 < g1) after = batched_ref(A, mask, mine, C, gi + 2);
        float2 *next_raw = raw + 256 * (buf ^ 1);
        batched_gate<NT>(sd, frag, cur.g, raw + 256 * buf, cur.m, tb, [&] {
            if (put1) next_raw[threadIdx.x] = e1;
        });
        cur = nxt;
        nxt = after;
        buf ^= 1;
    }
}

// One operation (k qubits; block position of its bit b in bits 3b..3b+2 of
// `lpp`) on a column of a fused block's matrix, as the host's fusion does
// it: for each group, w_j = sum_l U[j][l] v_l in FP64 with the complex
// products and sums rounded one by one (no contraction into FMAs).
__device__ __forceinline__ int member_spread(int j, int k, int lpp) {
    int x = 0;
    for (int b = 0; b < k; ++b) x |= ((j >> b) & 1) << ((lpp >> (3 * b)) & 7);
    return x;
}

__device__ __forceinline__ int member_base(int grp, int opmask) {
    int base = 0, rest = grp;  // the group's bits, in order, at the positions the operation leaves free
    for (int p = 0; p < kMaxGateQubits; ++p)
        if (!((opmask >> p) & 1)) {
            base |= (rest & 1) << p;
            rest >>= 1;
        }
    return base;
}

// k <= 3: the group's v in registers, U an LDS copy.
template <int K>
__device__ __forceinline__ void fuse_member_small(double2 *col, int D, int lpp, const double2 *U) {
#pragma clang fp contract(off)
    constexpr int d = 1 << K;
    int opmask = 0, off[d];
#pragma unroll
    for (int b = 0; b < K; ++b) opmask |= 1 << ((lpp >> (3 * b)) & 7);
#pragma unroll
    for (int j = 0; j < d; ++j) off[j] = member_spread(j, K, lpp);
    for (int grp = 0; grp < (D >> K); ++grp) {
        const int base = member_base(grp, opmask);
        double2 v[d];
#pragma unroll
        for (int l = 0; l < d; ++l) v[l] = col[base + off[l]];
#pragma unroll
        for (int j = 0; j < d; ++j) {
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int l = 0; l < d; ++l) {
                const double2 u = U[j * d + l];
                const double pr = u.x * v[l].x - u.y * v[l].y;
                const double pi = u.x * v[l].y + u.y * v[l].x;
                sr = sr + pr;
                si = si + pi;
            }
            col[base + off[j]] = make_double2(sr, si);
        }
    }
}

// k = 4, 5 (a wide gate sharing a block with a channel): v from `old`, a
// copy of the column taken before the operation, U from global memory.
__device__ __forceinline__ void fuse_member_wide(double2 *col, double2 *old, int D, int k, int lpp,
                                                 const double2 *U) {
#pragma clang fp contract(off)
    const int d = 1 << k;
    for (int r = 0; r < D; ++r) old[r] = col[r];
    int opmask = 0;
    for (int b = 0; b < k; ++b) opmask |= 1 << ((lpp >> (3 * b)) & 7);
    for (int grp = 0; grp < (D >> k); ++grp) {
        const int base = member_base(grp, opmask);
        for (int j = 0; j < d; ++j) {
            double sr = 0.0, si = 0.0;
            for (int l = 0; l < d; ++l) {
                const double2 u = U[j * d + l];
                const double2 v = old[base + member_spread(l, k, lpp)];
                const double pr = u.x * v.x - u.y * v.y;
                const double pi = u.x * v.y + u.y * v.x;
                sr = sr + pr;
                si = si + pi;
            }
            col[base + member_spread(j, k, lpp)] = make_double2(sr, si);
        }
    }
}

// The matrix of block `rel` of the job's circuit with the job's picks, by
// one wavefront: each active lane carries one column of the product from
// the identity through the block's operations in order, in the wavefront's
// LDS workspace `ws` (1024 complex128: the column and its copy, so 32
// columns at a time for k <= 4 and 16 for k = 5; operators of up to 3
// qubits are staged in `ush`, 64 complex128), and writes it as complex64
// to the job's copy of the block's matrix.  Channel picks are drawn again
// (the same Philox call as the draw pass).
__device__ __forceinline__ void fuse_patched(const BatchArgs &A, const BatchJob &J, const BatchCircuit &C,
                                             int rel, double2 *ws, double2 *ush, float2 *mine) {
    const BatchGate g = A.gates[C.g0 + rel];
    const int D = 1 << g.k;
    const int per_pass = D <= 16 ? D : 16;
    const int lane = int(threadIdx.x) & 63;
    double2 *col = ws + lane * D;
    double2 *old = ws + 512 + lane * D;
    for (int c0 = 0; c0 < D; c0 += per_pass) {
        const bool on = lane < per_pass;
        const int c = c0 + lane;
        if (on)
            for (int r = 0; r < D; ++r) col[r] = make_double2(r == c ? 1.0 : 0.0, 0.0);
        for (int mi = g.m0; mi < g.m1; ++mi) {
            const BatchMember M = A.members[mi];
            const double2 *U;
            if (M.src >= 0) {
                U = A.fmats + M.src;
            } else {
                const int ci = -M.src - 1;
                const BatchChannel ch = A.chans[C.ch0 + ci];
                const int pick = draw_pick(A.pbar + ch.pbar, ch.nk,
                                           philox_uniform(J.seed, uint32_t(ci), J.traj, J.circ_id, kStreamChannel));
                if ((ch.identity >> pick) & 1u) continue;
                U = A.fmats + ch.unit + pick * (1 << (2 * M.k));
            }
            int lpp = 0;
#pragma unroll
            for (int b = 0; b < kMaxGateQubits; ++b) lpp |= (M.lp[b] & 7) << (3 * b);
            if (M.k <= 3) {
                // the wavefront's lanes run in lockstep: the previous
                // operator's reads precede these writes, and these writes
                // precede the reads below
                __builtin_amdgcn_wave_barrier();
                if (lane < (1 << (2 * M.k))) ush[lane] = U[lane];
                __builtin_amdgcn_wave_barrier();
                if (on) {
                    if (M.k == 1) fuse_member_small<1>(col, D, lpp, ush);
                    else if (M.k == 2) fuse_member_small<2>(col, D, lpp, ush);
                    else fuse_member_small<3>(col, D, lpp, ush);
                }
            } else if (on) {
                fuse_member_wide(col, old, D, M.k, lpp, U);
            }
        }
        if (on) {
            float2 *dst = mine + (g.mat - C.pool0);
            for (int r = 0; r < D; ++r) dst[r * D + c] = make_float2(float(col[r].x), float(col[r].y));
        }
    }
}

// Persistent launch: each workgroup takes jobs blockIdx.x, + gridDim.x, ...
// A job is one trajectory: its channels are drawn, the blocks its picks
// change are rebuilt, the state starts as |0...0>, the circuit's blocks run
// with the job's matrices, and the workgroup samples the final state
// (inverse CDF over 256 contiguous chunks whose FP64 sums are scanned in a
// fixed order; readout flips as in sample_draw).
template <int NT>
__global__ __launch_bounds__(NT) void run_batched(BatchArgs A) {
    constexpr int LNT = ilog2(NT);
    extern __shared__ float2 smem[];
    float2 *sd = smem;                                                   // 2^13 amplitudes
    float *frag = reinterpret_cast<float *>(smem + (1 << kBatchLdsQubits));  // 2048 floats
    float2 *raw = smem + (1 << kBatchLdsQubits) + 1024;                  // 2 x 256 entries
    __shared__ double part[kBlock];
    float2 *slot = A.slots ? A.slots + size_t(blockIdx.x) * size_t(A.slot_amps) : nullptr;
    float2 *mine = A.patched + size_t(blockIdx.x) * size_t(A.patched_stride);
    uint32_t *mask = reinterpret_cast<uint32_t *>(part);  // blocks the job's picks change
    for (int job = blockIdx.x; job < A.n_jobs; job += gridDim.x) {
        const BatchJob J = A.jobs[job];
        const BatchCircuit C = A.circs[J.circuit];
        const int n = C.n;
        const int dim = 1 << n;
        // the job's channel draws (one Philox call per channel, Algorithm
        // 2's fast path), recorded when asked; a pick other than the default
        // one flags its block
        const int words = (C.n_gates + 31) >> 5;
        for (int w = threadIdx.x; w < words; w += NT) mask[w] = 0u;
        __syncthreads();
        for (int c = threadIdx.x; c < C.nch; c += NT) {
            const BatchChannel ch = A.chans[C.ch0 + c];
            const int pick = draw_pick(A.pbar + ch.pbar, ch.nk,
                                       philox_uniform(J.seed, uint32_t(c), J.traj, J.circ_id, kStreamChannel));
            if (J.choices >= 0) A.choices[J.choices + c] = int8_t(pick);
            if (pick != ch.default_pick) atomicOr(&mask[ch.gate >> 5], 1u << (ch.gate & 31));
        }
        __syncthreads();
        // the flagged blocks' matrices with the job's picks, one wavefront
        // per block, by the first four wavefronts (workspace: a quarter of
        // the LDS state area each)
        {
            const int wave = int(threadIdx.x) >> 6;
            double2 *ws = reinterpret_cast<double2 *>(sd) + wave * 1024;
            double2 *ush = reinterpret_cast<double2 *>(raw) + wave * 64;
            for (int w = wave; wave < 4 && w < words; w += 4) {
                uint32_t bits = __builtin_amdgcn_readfirstlane(mask[w]);
                while (bits) {
                    const int b = __builtin_ctz(bits);
                    bits &= bits - 1u;
                    fuse_patched(A, J, C, 32 * w + b, ws, ush, mine);
                }
            }
            // The workgroup's own global stores (these copies, the state slot)
            // are read back only by its own wavefronts, which share one CU and
            // its L1: the barrier's workgroup-scope ordering suffices, and no
            // device-scope fence (an L2 write-back and invalidate on gfx950)
            // is needed anywhere in this kernel.
            __syncthreads();
        }
        // the state: LDS (resident) or the workgroup's slot, each accessed
        // through its own pointer so that LDS accesses stay LDS instructions
        const bool res = C.resident != 0;
        for (int i = threadIdx.x; i < dim; i += NT) {
            const float2 z = make_float2(i == 0 ? 1.f : 0.f, 0.f);
            if (res) sd[i] = z;
            else slot[i] = z;
        }
        __syncthreads();
        for (int si = C.s0; si < C.s1; ++si) {
            const BatchSweep &S = A.sweeps[si];
            if (C.resident) {
                batched_blocks<NT>(A, mask, mine, C, S.g0, S.g1, sd, frag, raw, n);
                continue;
            }
            // tiled: one pass over the slot, tile by tile
            const int tb = S.tb;
            const int R = (1 << tb) / NT;
            int off_tid = 0;
            for (int b = 0; b < LNT; ++b)
                if ((threadIdx.x >> b) & 1) off_tid |= 1 << S.pos[b];
            const int n_tiles = dim >> tb;
            for (int t = 0; t < n_tiles; ++t) {
                int base = t;
                for (int b = 0; b < tb; ++b) {
                    const int q = S.pos[b];
                    base = ((base >> q) << (q + 1)) | (base & ((1 << q) - 1));
                }
                base += off_tid;
                for (int r = 0; r < R; ++r) {
                    int o = 0;
                    for (int b = LNT; b < tb; ++b)
                        if (((r << LNT) >> b) & 1) o |= 1 << S.pos[b];
                    sd[threadIdx.x + (r << LNT)] = slot[base + o];
                }
                __syncthreads();
                batched_blocks<NT>(A, mask, mine, C, S.g0, S.g1, sd, frag, raw, tb);
                for (int r = 0; r < R; ++r) {
                    int o = 0;
                    for (int b = LNT; b < tb; ++b)
                        if (((r << LNT) >> b) & 1) o |= 1 << S.pos[b];
                    slot[base + o] = sd[threadIdx.x + (r << LNT)];
                }
                __syncthreads();
            }
        }
        // sampling: chunk c = amplitudes [c*L, (c+1)*L), L = dim / 256 (>= 1),
        // the same 256 chunks at either group size
        const int L = dim >= kBlock ? dim / kBlock : 1;
        const int chunks = dim >= kBlock ? kBlock : dim;
        auto chunk_sum = [&](const float2 *p) {
            double acc = 0.0;
            for (int i = 0; i < L; ++i) {
                const float2 v = p[threadIdx.x * L + i];
                acc = fma(double(v.x), double(v.x), fma(double(v.y), double(v.y), acc));
            }
            return acc;
        };
        double acc = 0.0;
        if (int(threadIdx.x) < chunks) acc = res ? chunk_sum(sd) : chunk_sum(slot);
        if (int(threadIdx.x) < kBlock) part[threadIdx.x] = acc;
        __syncthreads();
        // inclusive prefix of the chunk sums by one wavefront: lane l sums
        // chunks 4l..4l+3 in order, the lanes' totals are scanned across
        // the wavefront, and chunk c's prefix is the lane's offset plus its
        // own running sum (a fixed order, so every launch rounds alike),
        // then made exactly non-decreasing by a running maximum (the two
        // summation orders can differ by an ulp where lanes meet)
        if (threadIdx.x < 64) {
            const int l = int(threadIdx.x);
            double p[4];
            double run = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                run += 4 * l + i < chunks ? part[4 * l + i] : 0.0;
                p[i] = run;
            }
            double t = run;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const double u = __shfl_up(t, o);
                if (l >= o) t += u;
            }
            double off = __shfl_up(t, 1);
            if (l == 0) off = 0.0;
            double hi = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                p[i] = fmax(hi, off + p[i]);
                hi = p[i];
            }
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const double u = __shfl_up(hi, o);
                if (l >= o) hi = fmax(hi, u);
            }
            double below = __shfl_up(hi, 1);
            if (l == 0) below = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (4 * l + i < chunks) part[4 * l + i] = fmax(below, p[i]);
        }
        __syncthreads();
        const double N = part[chunks - 1];
        for (int smp = threadIdx.x; smp < C.n_samples; smp += NT) {
            const double target = philox_uniform(J.seed, uint32_t(smp), J.traj, J.circ_id, kStreamMeasure) * N;
            int lo = 0, hi = chunks;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (target < part[mid]) hi = mid; else lo = mid + 1;
            }
            uint32_t x;
            if (lo >= chunks) {
                x = uint32_t(dim - 1);
            } else {
                auto within = [&](const float2 *p) {
                    double run = lo > 0 ? part[lo - 1] : 0.0;
                    for (int i = 0; i < L; ++i) {
                        const float2 v = p[lo * L + i];
                        run += fma(double(v.x), double(v.x), double(v.y) * double(v.y));
                        if (target < run) return i;
                    }
                    return L - 1;
                };
                x = uint32_t(lo * L + (res ? within(sd) : within(slot)));
            }
            if (C.readout >= 0) {
                const double *e0 = A.readout + C.readout;
                const double *e1 = e0 + n;
                for (int q = 0; q < n; ++q) {
                    const int bit = int((x >> q) & 1u);
                    const double u = philox_uniform(J.seed, uint32_t(smp * n + q), J.traj, J.circ_id,
                                                    kStreamReadout);
                    if (u < (bit ? e1[q] : e0[q])) x ^= 1u << q;
                }
            }
            A.out[J.out + smp] = x;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- utility

template <typename Idx>
__global__ __launch_bounds__(kBlock) void set_basis(float2 *__restrict__ amp, Idx dim, Idx index) {
    const Idx stride = Idx(gridDim.x) * Idx(kBlock);
    for (Idx i = Idx(blockIdx.x) * Idx(kBlock) + Idx(threadIdx.x); i < dim; i += stride)
        amp[i] = make_float2(i == index ? 1.f : 0.f, 0.f);
}

// A state copy: pairs of amplitudes as 16-byte loads and stores, over a
// grid of four 256-work-item groups per CU (the shape that copied a 2 GiB
// state fastest in a sweep of grids and unrolling).
__global__ __launch_bounds__(kBlock) void copy_pairs(float4 *__restrict__ dst, const float4 *__restrict__ src,
                                                     int64_t pairs) {
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < pairs; i += stride) dst[i] = src[i];
}

template <typename Idx>
__global__ __launch_bounds__(kBlock) void scale_state(float2 *__restrict__ amp, Idx dim, float s) {
    const Idx stride = Idx(gridDim.x) * Idx(kBlock);
    for (Idx i = Idx(blockIdx.x) * Idx(kBlock) + Idx(threadIdx.x); i < dim; i += stride) {
        float2 v = amp[i];
        amp[i] = make_float2(v.x * s, v.y * s);
    }
}

// ---------------------------------------------------------------- reductions

// Fixed-order workgroup sum of W per-thread values; thread 0 writes them.
template <int W>
__device__ __forceinline__ void block_sum_write(double (&vals)[W], double *__restrict__ dst) {
    __shared__ double red[kBlock / 64][W];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        double x = vals[w];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        vals[w] = x;
    }
    if (lane == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) red[wave][w] = vals[w];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            double s = red[0][w];
#pragma unroll
            for (int i = 1; i < kBlock / 64; ++i) s += red[i][w];
            dst[w] = s;
        }
    }
}

template <typename Idx>
__global__ __launch_bounds__(kBlock) void norm_partials(const float2 *__restrict__ amp, Idx dim,
                                                        double *__restrict__ partials) {
    double acc[1] = {0.0};
    const Idx stride = Idx(gridDim.x) * Idx(kBlock);
    for (Idx i = Idx(blockIdx.x) * Idx(kBlock) + Idx(threadIdx.x); i < dim; i += stride) {
        const float2 v = amp[i];
        const double re = v.x, im = v.y;
        acc[0] = fma(re, re, fma(im, im, acc[0]));
    }
    block_sum_write<1>(acc, partials + blockIdx.x);
}

template <int K, typename Idx>
__global__ __launch_bounds__(kBlock) void rdm_partials(const float2 *__restrict__ amp, Idx groups,
                                                       TargetArgs ta,
                                                       double *__restrict__ partials) {
    constexpr int D = 1 << K;
    constexpr int W = 2 * D * D;
    double acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = 0.0;
    const Idx stride = Idx(gridDim.x) * Idx(kBlock);
    for (Idx g = Idx(blockIdx.x) * Idx(kBlock) + Idx(threadIdx.x); g < groups; g += stride) {
        const Idx base = spread_index<K, Idx>(g, ta.t);
        double vr[D], vi[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const float2 v = amp[base + local_offset<K, Idx>(j, ta.t)];
            vr[j] = v.x;
            vi[j] = v.y;
        }
        // R[j][l] += v_j conj(v_l)
#pragma unroll
        for (int j = 0; j < D; ++j)
#pragma unroll
            for (int l = 0; l < D; ++l) {
                acc[2 * (j * D + l)] = fma(vr[j], vr[l], fma(vi[j], vi[l], acc[2 * (j * D + l)]));
                acc[2 * (j * D + l) + 1] =
                    fma(vi[j], vr[l], fma(-vr[j], vi[l], acc[2 * (j * D + l) + 1]));
            }
    }
    block_sum_write<W>(acc, partials + size_t(blockIdx.x) * W);
}

template <int K, typename Idx>
__global__ __launch_bounds__(kBlock) void apply_copy_norm(const float2 *__restrict__ in,
                                                          float2 *__restrict__ out, Idx groups,
                                                          GateArgs<K> a,
                                                          double *__restrict__ partials) {
    constexpr int D = 1 << K;
    double acc[2] = {0.0, 0.0};
    const Idx stride = Idx(gridDim.x) * Idx(kBlock);
    for (Idx g = Idx(blockIdx.x) * Idx(kBlock) + Idx(threadIdx.x); g < groups; g += stride) {
        const Idx base = spread_index<K, Idx>(g, a.t);
        float2 v[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            v[j] = in[base + local_offset<K, Idx>(j, a.t)];
            acc[1] = fma(double(v[j].x), double(v[j].x), fma(double(v[j].y), double(v[j].y), acc[1]));
        }
#pragma unroll
        for (int j = 0; j < D; ++j) {
            float2 w = make_float2(0.f, 0.f);
#pragma unroll
            for (int l = 0; l < D; ++l) w = cmac(w, a.m[j * D + l], v[l]);
            out[base + local_offset<K, Idx>(j, a.t)] = w;
            acc[0] = fma(double(w.x), double(w.x), fma(double(w.y), double(w.y), acc[0]));
        }
    }
    block_sum_write<2>(acc, partials + size_t(blockIdx.x) * 2);
}

// Per-qubit weights (see launch_zweights).  Workgroup w owns the contiguous
// chunk [w 2^c, (w + 1) 2^c); work-item t reads x = chunk + 256 i + t, so
// bits 0..7 of x come from t, bits 8..c-1 from the iteration i (uniform) and
// the rest from the chunk (uniform per workgroup).  A work-item keeps its
// total and one sum per iteration bit; the record's entries follow from
// those (bit q < 8: the work-item's total if its bit q is set).
constexpr int kZIterBits = 16;
template <typename Idx>
__global__ __launch_bounds__(kBlock) void zweight_partials(const float2 *__restrict__ amp, int n, int c,
                                                           double *__restrict__ partials) {
    const int t = threadIdx.x;
    const int ibits = c > 8 ? c - 8 : 0;
    const Idx chunk = Idx(blockIdx.x) << c;
    const Idx iters = Idx(1) << ibits;
    const int active = c >= 8 || t < (1 << c);
    double tot = 0.0;
    double per_bit[kZIterBits];
#pragma unroll
    for (int j = 0; j < kZIterBits; ++j) per_bit[j] = 0.0;
    if (active) {
        for (Idx i = 0; i < iters; ++i) {
            const float2 v = amp[chunk + (i << 8) + Idx(t)];
            const double p = fma(double(v.x), double(v.x), double(v.y) * double(v.y));
            tot += p;
#pragma unroll
            for (int j = 0; j < kZIterBits; ++j)
                if (j < ibits && ((i >> j) & 1)) per_bit[j] += p;
        }
    }
    double vals[kZRecord];
    vals[0] = tot;
#pragma unroll
    for (int q = 0; q < kZRecord - 1; ++q) {
        double x = 0.0;
        if (q < n) {
            if (q < 8) x = ((t >> q) & 1) ? tot : 0.0;
            else if (q < 8 + ibits) x = per_bit[q - 8];
            else x = ((chunk >> q) & 1) ? tot : 0.0;
        }
        vals[1 + q] = x;
    }
    block_sum_write<kZRecord>(vals, partials + size_t(blockIdx.x) * kZRecord);
}

// Sum `count` records of `width` doubles in a fixed order (one workgroup).
__global__ __launch_bounds__(kBlock) void reduce_records(const double *__restrict__ partials,
                                                         int count, int width,
                                                         double *__restrict__ out) {
    __shared__ double red[kBlock];
    for (int w = 0; w < width; ++w) {
        double s = 0.0;
        for (int i = threadIdx.x; i < count; i += kBlock) s += partials[size_t(i) * width + w];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = kBlock / 2; h >= 1; h >>= 1) {
            if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[w] = red[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- sampling

// Per-lane sum of |amp|^2 over `per` consecutive amplitudes starting at
// `first`, in index order (pairs loaded as one 16-byte access).
template <typename Idx>
__device__ __forceinline__ double chunk_weight(const float2 *__restrict__ amp, Idx first, int per) {
    double acc = 0.0;
    if (per >= 2) {
        const float4 *p4 = reinterpret_cast<const float4 *>(amp + first);
        for (int i = 0; i < per / 2; ++i) {
            const float4 v = p4[i];
            acc = fma(double(v.x), double(v.x), fma(double(v.y), double(v.y), acc));
            acc = fma(double(v.z), double(v.z), fma(double(v.w), double(v.w), acc));
        }
    } else {
        const float2 v = amp[first];
        acc = fma(double(v.x), double(v.x), double(v.y) * double(v.y));
    }
    return acc;
}

// One wavefront per sampling block of 2^B amplitudes (kBlock / 64 blocks per
// workgroup): the lanes read the block coalesced (lane j takes pairs j,
// j + 64, ... as 16-byte loads) and add in that fixed order, then a fixed
// shuffle tree adds the lanes.
template <typename Idx>
__global__ __launch_bounds__(kBlock) void sample_block_sums(const float2 *__restrict__ amp, int B,
                                                            int64_t nb, double *__restrict__ sums) {
    const int64_t blk = int64_t(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (blk >= nb) return;  // uniform over the wavefront
    const int len = 1 << B;
    const Idx first = Idx(blk) << B;
    double x = 0.0;
    if (len >= 128) {
        const float4 *p4 = reinterpret_cast<const float4 *>(amp + first);
#pragma unroll 8
        for (int i = lane; i < len / 2; i += 64) {
            const float4 v = p4[i];
            x = fma(double(v.x), double(v.x), fma(double(v.y), double(v.y), x));
            x = fma(double(v.z), double(v.z), fma(double(v.w), double(v.w), x));
        }
    } else {
        for (int i = lane; i < len; i += 64) {
            const float2 v = amp[first + Idx(i)];
            x = fma(double(v.x), double(v.x), fma(double(v.y), double(v.y), x));
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) sums[blk] = x;
}

// Inclusive prefix of the block sums in index order, in three fixed-order
// steps: every tile of kScanThreads * kScanPer sums is scanned by its own
// workgroup; one workgroup scans the tile totals into exclusive tile offsets
// (written over the block sums, which are no longer needed) and the total;
// the offsets are added to the tiles after the first.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;
__device__ __forceinline__ double wave_inclusive_scan(double x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive prefix over the workgroup's kScanThreads values in thread order
// (wavefront scans, then the wavefront totals in order); *all gets the total.
__device__ __forceinline__ double workgroup_exclusive_scan(double x, double *wave_tot, double *all) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double inc = wave_inclusive_scan(x);
    if (lane == 63) wave_tot[wave] = inc;
    __syncthreads();
    double before = 0.0, sum = 0.0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wave) before += wave_tot[w];
        sum += wave_tot[w];
    }
    *all = sum;
    return before + (inc - x);
}

// A tile is loaded coalesced into LDS (one pad slot per kScanPer, so each
// work-item's run of kScanPer consecutive sums sits on distinct banks), each
// work-item adds its run, the runs' offsets come from one workgroup scan,
// and the runs' prefixes go back through LDS and out coalesced.
__device__ __forceinline__ int scan_slot(int i) { return i + i / kScanPer; }

__global__ __launch_bounds__(kScanThreads) void sample_scan_tiles(const double *__restrict__ sums,
                                                                  int64_t nb, double *__restrict__ incl) {
    __shared__ double tile[kScanTile + kScanTile / kScanPer];
    __shared__ double wave_tot[kScanThreads / 64];
    const int t = threadIdx.x;
    const int64_t base = int64_t(blockIdx.x) * kScanTile;
    const int len = nb - base < kScanTile ? int(nb - base) : kScanTile;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int i = j * kScanThreads + t;
        tile[scan_slot(i)] = i < len ? sums[base + i] : 0.0;
    }
    __syncthreads();
    double v[kScanPer], tot = 0.0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = tile[scan_slot(t * kScanPer + j)];
        tot += v[j];
    }
    double all;
    double run = workgroup_exclusive_scan(tot, wave_tot, &all);
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        run += v[j];
        tile[scan_slot(t * kScanPer + j)] = run;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int i = j * kScanThreads + t;
        if (i < len) incl[base + i] = tile[scan_slot(i)];
    }
}

// Tile totals (each tile's last prefix) added one after another: offsets[t]
// is the running sum before tile t, so that a tile's last prefix plus its
// offset equals the next offset exactly and the prefix stays non-decreasing
// across tiles.  *norm is the final sum.
constexpr int kScanMaxTiles = 2048;  // 2^(kMaxQubits - kSampleBlockBits) / kScanTile
__global__ __launch_bounds__(kScanThreads) void sample_scan_offsets(const double *__restrict__ incl,
                                                                    int64_t nb, int n_tiles,
                                                                    double *__restrict__ offsets,
                                                                    double *__restrict__ norm) {
    __shared__ double tot[kScanMaxTiles];
    for (int t = threadIdx.x; t < n_tiles; t += kScanThreads) {
        const int64_t end = int64_t(t + 1) * kScanTile;
        tot[t] = incl[(end < nb ? end : nb) - 1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int t0 = 0; t0 < n_tiles; t0 += 16) {
            double v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = t0 + j < n_tiles ? tot[t0 + j] : 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (t0 + j < n_tiles) {
                    offsets[t0 + j] = run;
                    run += v[j];
                }
        }
        *norm = run;
    }
}

__global__ __launch_bounds__(kBlock) void sample_scan_add(double *__restrict__ incl, int64_t nb,
                                                          const double *__restrict__ offsets) {
    const int64_t i = int64_t(kScanTile) + int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < nb) incl[i] += offsets[i / kScanTile];
}

// One wavefront per sample: find the block by a 64-way search over the block
// prefix, then the lanes sum 2^B/64 consecutive amplitudes each, scan those
// partial sums in a fixed order, and the first lane whose running sum passes
// the target walks its own amplitudes.  PER > 0: blocks of 64 * PER
// amplitudes, each lane's run kept in registers for the walk; PER = 0: any
// block size, the walk reloads.
template <typename Idx, int PER>
__global__ __launch_bounds__(kBlock) void sample_draw(const float2 *__restrict__ amp, int n, int B,
                                                      const double *__restrict__ incl, int64_t nb,
                                                      const double *__restrict__ norm,
                                                      uint64_t seed, uint32_t traj, uint32_t circ,
                                                      int n_samples, ReadoutDesc ro,
                                                      uint64_t *__restrict__ out) {
    const int s = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= n_samples) return;  // uniform over the wavefront
    const double N = *norm;
    const double target = philox_uniform(seed, uint32_t(s), traj, circ, kStreamMeasure) * N;
    // smallest block b with target < incl[b] (nb if none): the lanes probe
    // evenly spaced entries and a ballot keeps the first passing interval.
    // Invariant: the answer lies in [lo, hi], and hi passes or is nb.
    int64_t lo = 0, hi = nb;
    while (lo < hi) {
        const int64_t span = hi - lo;
        const int64_t step = span <= 64 ? 1 : (span + 63) / 64;
        int64_t probe = lo + int64_t(lane + 1) * step - 1;
        if (probe > hi - 1) probe = hi - 1;
        const bool pass = target < incl[probe];
        const uint64_t mask = __ballot(pass);
        if (mask == 0) {  // every probe up to hi - 1 fails
            lo = hi;
            break;
        }
        const int L = __ffsll((unsigned long long)mask) - 1;
        const int64_t pL = __shfl(probe, L, 64);
        const int64_t pprev = L > 0 ? __shfl(probe, L - 1, 64) : lo - 1;
        if (step == 1) {
            lo = pL;
            break;
        }
        lo = pprev + 1;
        hi = pL;
    }
    uint64_t x;
    if (lo >= nb) {
        x = (uint64_t(1) << n) - 1;
    } else {
        const double base = lo > 0 ? incl[lo - 1] : 0.0;
        const Idx first = Idx(lo) << B;
        const int len = 1 << B;
        const int per = PER > 0 ? PER : (len >= 64 ? len / 64 : 1);
        const int lanes = len >= 64 ? 64 : len;
        double part = 0.0;
        float4 keep[PER > 0 ? PER / 2 : 1];
        if constexpr (PER > 0) {
            const float4 *p4 = reinterpret_cast<const float4 *>(amp + first + Idx(lane * PER));
#pragma unroll
            for (int i = 0; i < PER / 2; ++i) keep[i] = p4[i];
#pragma unroll
            for (int i = 0; i < PER / 2; ++i) {
                part = fma(double(keep[i].x), double(keep[i].x), fma(double(keep[i].y), double(keep[i].y), part));
                part = fma(double(keep[i].z), double(keep[i].z), fma(double(keep[i].w), double(keep[i].w), part));
            }
        } else if (lane < lanes) {
            part = chunk_weight(amp, first + Idx(lane * per), per);
        }
        const double inc = base + wave_inclusive_scan(part);
        const uint64_t passed = __ballot(lane < lanes && target < inc);
        int pick = len - 1;
        if (passed) {
            const int L = __ffsll((unsigned long long)passed) - 1;
            // lane L walks its amplitudes from its exclusive prefix, adding
            // them as chunk_weight does
            int idx = L * per + per - 1;
            if (lane == L) {
                double run = inc - part;
                if constexpr (PER > 0) {
                    bool found = false;
#pragma unroll
                    for (int i = 0; i < PER / 2; ++i) {
                        const double r0 = fma(double(keep[i].x), double(keep[i].x),
                                              fma(double(keep[i].y), double(keep[i].y), run));
                        const double r1 = fma(double(keep[i].z), double(keep[i].z),
                                              fma(double(keep[i].w), double(keep[i].w), r0));
                        if (!found && target < r0) {
                            idx = L * PER + 2 * i;
                            found = true;
                        } else if (!found && target < r1) {
                            idx = L * PER + 2 * i + 1;
                            found = true;
                        }
                        run = r1;
                    }
                } else if (per >= 2) {
                    const float4 *p4 = reinterpret_cast<const float4 *>(amp + first + Idx(L * per));
                    for (int i = 0; i < per / 2; ++i) {
                        const float4 v = p4[i];
                        const double r0 = fma(double(v.x), double(v.x), fma(double(v.y), double(v.y), run));
                        if (target < r0) { idx = L * per + 2 * i; break; }
                        const double r1 = fma(double(v.z), double(v.z), fma(double(v.w), double(v.w), r0));
                        if (target < r1) { idx = L * per + 2 * i + 1; break; }
                        run = r1;
                    }
                } else {
                    idx = L;
                }
            }
            pick = __shfl(idx, L, 64);
        }
        x = uint64_t(first) + uint64_t(pick);
    }
    if (lane == 0) {
        if (ro.enabled) {
            for (int q = 0; q < n; ++q) {
                const int bit = int((x >> q) & 1u);
                const double u = philox_uniform(seed, uint32_t(uint64_t(s) * uint64_t(n) + uint64_t(q)),
                                                traj, circ, kStreamReadout);
                if (u < (bit ? ro.e1[q] : ro.e0[q])) x ^= uint64_t(1) << q;
            }
        }
        out[s] = x;
    }
}

// ---------------------------------------------------------------- helpers

inline unsigned grid_for(uint64_t work_items, unsigned cap = 1u << 20) {
    uint64_t b = (work_items + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return unsigned(b);
}

template <int K>
GateArgs<K> make_args(const GateDesc &g) {
    GateArgs<K> a;
    constexpr int D = 1 << K;
    for (int i = 0; i < D * D; ++i) a.m[i] = g.m[i];
    for (int b = 0; b < K; ++b) a.t[b] = g.t[b];
    return a;
}

template <typename Idx>
hipError_t apply_direct_idx(float2 *amp, int n, const GateDesc &g, const float2 *mat_dev,
                            hipStream_t st) {
    const Idx groups = Idx(1) << (n - g.k);
    const unsigned grid = grid_for(uint64_t(groups));
    TargetArgs ta;
    for (int b = 0; b < kMaxGateQubits; ++b) ta.t[b] = b < g.k ? g.t[b] : 0;
    switch (g.k) {
        case 1: apply_direct<1, Idx><<<grid, kBlock, 0, st>>>(amp, groups, mat_dev, ta); break;
        case 2: apply_direct<2, Idx><<<grid, kBlock, 0, st>>>(amp, groups, mat_dev, ta); break;
        case 3: apply_direct<3, Idx><<<grid, kBlock, 0, st>>>(amp, groups, mat_dev, ta); break;
        case 4: apply_direct<4, Idx><<<grid, kBlock, 0, st>>>(amp, groups, mat_dev, ta); break;
        case 5: apply_direct<5, Idx><<<grid, kBlock, 0, st>>>(amp, groups, mat_dev, ta); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int device_cus() {
    // initialised once, thread-safely (several host threads may launch at once)
    static const int cus = [] {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            c = 256;
        return c;
    }();
    return cus;
}

// Once per instantiation, thread-safely: allow the matrix region, and read
// how many workgroups per CU registers and waves allow (with no matrices the
// LDS is not what limits the count); a negative value is an error.
template <int TB, typename Idx, bool K5, int NT, bool RK>
int tile_reg_limit() {
    static const int reg_limit = [] {
        const void *fn = reinterpret_cast<const void *>(&apply_tile<TB, Idx, K5, NT, RK>);
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                int(sizeof(float2) * kTileMatBudget)) != hipSuccess)
            return -1;
        int blocks = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, NT, 0) != hipSuccess) return -1;
        return blocks < 1 ? 1 : blocks;
    }();
    return reg_limit;
}

// launch = false only sets the instantiation up (no stream work), so that a
// later launch under stream capture makes no attribute or occupancy calls.
template <int TB, typename Idx, bool K5, int NT, bool RK>
hipError_t tile_launch(float2 *amp, int n, const TileArgs &a, hipStream_t st, bool launch,
                       int *grid_out) {
    // static tile + dynamic matrices
    const size_t dyn = sizeof(float2) * size_t(a.mat_total);
    const size_t lds = sizeof(float2) * (size_t(1) << TB) + dyn;
    const int reg_limit = tile_reg_limit<TB, Idx, K5, NT, RK>();
    if (reg_limit < 0) return hipErrorInvalidDeviceFunction;
    const int cus = device_cus();
    if (!launch) return hipSuccess;
    const Idx n_tiles = Idx(1) << (n - TB);
    // persistent grid: as many workgroups as are resident at once at this LDS size
    int per_cu = int((160u * 1024u) / lds);
    if (per_cu < 1) per_cu = 1;
    if (per_cu > reg_limit) per_cu = reg_limit;
    uint64_t grid = uint64_t(cus) * uint64_t(per_cu);
    if (grid > uint64_t(n_tiles)) grid = uint64_t(n_tiles);
    if (RK && grid > uint64_t(kMaxReduceBlocks)) return hipErrorInvalidValue;  // record space
    if (grid_out) *grid_out = int(grid);
    apply_tile<TB, Idx, K5, NT, RK><<<unsigned(grid), NT, dyn, st>>>(amp, n_tiles, a);
    return hipGetLastError();
}

template <int TB, typename Idx>
hipError_t tile_launch_k(float2 *amp, int n, const TileArgs &a, hipStream_t st, bool launch,
                         int *grid_out) {
    bool k5 = false;
    for (int gi = 0; gi < a.n_gates; ++gi) k5 |= a.g[gi].k == 5;
    // Four wavefronts per SIMD hide the LDS and MFMA latency: a 2^14-amplitude
    // tile (128 KiB) leaves room for one workgroup per CU, so it runs 1024
    // work-items; 2^13 (64 KiB) for two, with 512 each.  Smaller tiles fit
    // more workgroups and do better with 256 (measured on the 24-qubit noisy
    // grid).
    constexpr int NT = TB >= 14 ? 1024 : (TB >= 13 ? 512 : kBlock);
    if (a.rdm_out) {
        if (k5) return hipErrorInvalidValue;
        return tile_launch<TB, Idx, false, NT, true>(amp, n, a, st, launch, grid_out);
    }
    return k5 ? tile_launch<TB, Idx, true, NT, false>(amp, n, a, st, launch, grid_out)
              : tile_launch<TB, Idx, false, NT, false>(amp, n, a, st, launch, grid_out);
}

template <typename Idx>
hipError_t apply_tile_idx(float2 *amp, int n, const TileArgs &a, hipStream_t st, bool launch,
                          int *grid_out) {
    switch (a.tb) {
        case 10: return tile_launch_k<10, Idx>(amp, n, a, st, launch, grid_out);
        case 11: return tile_launch_k<11, Idx>(amp, n, a, st, launch, grid_out);
        case 12: return tile_launch_k<12, Idx>(amp, n, a, st, launch, grid_out);
        case 13: return tile_launch_k<13, Idx>(amp, n, a, st, launch, grid_out);
        case 14: return tile_launch_k<14, Idx>(amp, n, a, st, launch, grid_out);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_select(const SelectArgs &a, hipStream_t st) {
    if (a.nk < 1 || a.D < 1 || a.Db < 1 || a.Db > 32) return hipErrorInvalidValue;
    select_branch<<<1, 64, 0, st>>>(a);
    return hipGetLastError();
}

int batched_grid() {
    const int per_cu = int((160u * 1024u) / (sizeof(float2) * ((1u << kBatchLdsQubits) + 1536u) +
                                             sizeof(double) * kBlock));
    return device_cus() * (per_cu < 1 ? 1 : per_cu);
}

// Launches with no more jobs than CUs run one 512-work-item group per job
// (eight wavefronts share each block's work, twice the 256-work-item
// form's); larger ones run two 256-work-item groups per CU.  The grid never
// exceeds batched_grid(), which sizes the per-workgroup buffers.
hipError_t launch_batched(const BatchArgs &a, int grid, hipStream_t st) {
    const size_t lds = sizeof(float2) * ((size_t(1) << kBatchLdsQubits) + 1536);
    static const hipError_t attr256 = hipFuncSetAttribute(reinterpret_cast<const void *>(&run_batched<256>),
                                                          hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    static const hipError_t attr512 = hipFuncSetAttribute(reinterpret_cast<const void *>(&run_batched<512>),
                                                          hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (attr256 != hipSuccess) return attr256;
    if (attr512 != hipSuccess) return attr512;
    if (grid < 1 || a.n_jobs < 1) return hipErrorInvalidValue;
    if (a.n_jobs <= device_cus() && a.n_jobs <= grid)
        run_batched<512><<<unsigned(a.n_jobs), 512, lds, st>>>(a);
    else
        run_batched<256><<<unsigned(grid), 256, lds, st>>>(a);
    return hipGetLastError();
}

int reduce_blocks_for(int n, int k) {
    // at least 4 groups per work-item; a fixed count per (n, k)
    const uint64_t groups = uint64_t(1) << (n - k);
    uint64_t b = groups / (4u * kBlock);
    if (b < 1) b = 1;
    if (b > kMaxReduceBlocks) b = kMaxReduceBlocks;
    return int(b);
}

hipError_t launch_set_basis(float2 *amp, int n, uint64_t index, hipStream_t st) {
    const uint64_t dim = uint64_t(1) << n;
    const unsigned grid = grid_for(dim);
    if (n <= 31)
        set_basis<uint32_t><<<grid, kBlock, 0, st>>>(amp, uint32_t(dim), uint32_t(index));
    else
        set_basis<uint64_t><<<grid, kBlock, 0, st>>>(amp, dim, index);
    return hipGetLastError();
}

hipError_t launch_copy_state(float2 *dst, const float2 *src, int n, hipStream_t st) {
    if (n < 1 || n > kMaxQubits || !dst || !src) return hipErrorInvalidValue;
    const int64_t pairs = int64_t(1) << (n - 1);
    const int64_t want = (pairs + kBlock - 1) / kBlock;
    const int64_t cap = int64_t(device_cus()) * 4;
    const unsigned grid = unsigned(want < cap ? want : cap);
    copy_pairs<<<grid, kBlock, 0, st>>>(reinterpret_cast<float4 *>(dst), reinterpret_cast<const float4 *>(src),
                                        pairs);
    return hipGetLastError();
}

hipError_t launch_scale(float2 *amp, int n, float s, hipStream_t st) {
    const uint64_t dim = uint64_t(1) << n;
    const unsigned grid = grid_for(dim);
    if (n <= 31)
        scale_state<uint32_t><<<grid, kBlock, 0, st>>>(amp, uint32_t(dim), s);
    else
        scale_state<uint64_t><<<grid, kBlock, 0, st>>>(amp, dim, s);
    return hipGetLastError();
}

bool tile_for_gate(int n, const GateDesc &g, TileArgs &a) {
    if (n < kTileMinQubits) return false;
    bool low = false;
    for (int b = 0; b < g.k; ++b) low |= g.t[b] < 6;
    if (!low) return false;
    bool in_tile[kMaxQubits] = {false};
    int cnt = 0;
    for (int q = 0; q < 6; ++q) { in_tile[q] = true; ++cnt; }
    for (int b = 0; b < g.k; ++b)
        if (!in_tile[g.t[b]]) { in_tile[g.t[b]] = true; ++cnt; }
    int tb = cnt;
    if (tb < 10) tb = 10;
    if (tb < g.k + 8) tb = g.k + 8;
    if (tb > n) tb = n;
    for (int q = 0; q < n && cnt < tb; ++q)
        if (!in_tile[q]) { in_tile[q] = true; ++cnt; }
    a.tb = tb;
    int i = 0;
    for (int q = 0; q < n; ++q)
        if (in_tile[q]) a.pos[i++] = q;
    a.n_gates = 1;
    a.init_zero = 0;
    a.mat_total = tile_mat_slots(g.k);
    a.g[0].k = g.k;
    a.g[0].lofs = 0;
    a.g[0].pad = 0;
    a.g[0].mat = nullptr;
    for (int b = 0; b < g.k; ++b) {
        int lp = 0;
        while (a.pos[lp] != g.t[b]) ++lp;
        a.g[0].lt[b] = lp;  // ascending because g.t is ascending
    }
    return true;
}

hipError_t launch_apply_gate(float2 *amp, int n, const GateDesc &g, const float2 *mat_dev,
                             hipStream_t st) {
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    if (tile_for_gate(n, g, a)) {
        a.g[0].mat = mat_dev;
        return launch_apply_tile(amp, n, a, st);
    }
    if (n <= 31) return apply_direct_idx<uint32_t>(amp, n, g, mat_dev, st);
    return apply_direct_idx<uint64_t>(amp, n, g, mat_dev, st);
}

hipError_t launch_apply_tile(float2 *amp, int n, const TileArgs &a, hipStream_t st, int *grid_out) {
    return launch_apply_tile_impl(amp, n, a, st, true, grid_out);
}

hipError_t prepare_apply_tile(int n, const TileArgs &a) {
    return launch_apply_tile_impl(nullptr, n, a, nullptr, false);
}

hipError_t launch_apply_tile_impl(float2 *amp, int n, const TileArgs &a, hipStream_t st, bool launch,
                                  int *grid_out) {
    if (a.tb < 10 || a.tb > kMaxTileBits || a.tb > n || a.n_gates < 0 ||
        a.n_gates > kMaxTileGates || a.mat_total < 0 || a.mat_total > kTileMatBudget)
        return hipErrorInvalidValue;
    if (a.rdm_out && (a.rdm_lt < 0 || a.rdm_lt >= a.tb)) return hipErrorInvalidValue;
    // tile bits: ascending global positions below n, the first kTileLowBits
    // of them bits 0.. (the pair loads need local bit 0 = global bit 0)
    for (int b = 0; b < a.tb; ++b)
        if (a.pos[b] < 0 || a.pos[b] >= n || (b > 0 && a.pos[b] <= a.pos[b - 1]) ||
            (b < kTileLowBits && a.pos[b] != b))
            return hipErrorInvalidValue;
    for (int gi = 0; gi < a.n_gates; ++gi) {
        const TileGate &g = a.g[gi];
        if (g.k < 1 || g.k > kMaxGateQubits || g.k > a.tb || !g.mat || g.lofs < 0 ||
            g.lofs + tile_mat_slots(g.k) > a.mat_total)
            return hipErrorInvalidValue;
        for (int b = 0; b < g.k; ++b)
            if (g.lt[b] < 0 || g.lt[b] >= a.tb || (b > 0 && g.lt[b] <= g.lt[b - 1]))
                return hipErrorInvalidValue;
    }
    // each gate's address table for the swizzled tile layout
    TileArgs b = a;
    for (int gi = 0; gi < b.n_gates; ++gi) {
        TileGate &g = b.g[gi];
        switch (g.k) {
            case 1: gate_tables<1, SwizzledTile>(g.lt, g.tab); break;
            case 2: gate_tables<2, SwizzledTile>(g.lt, g.tab); break;
            case 3: gate_tables<3, SwizzledTile>(g.lt, g.tab); break;
            case 4: gate_tables<4, SwizzledTile>(g.lt, g.tab); break;
            default: gate_tables<5, SwizzledTile>(g.lt, g.tab); break;
        }
    }
    if (n <= 31) return apply_tile_idx<uint32_t>(amp, n, b, st, launch, grid_out);
    return apply_tile_idx<uint64_t>(amp, n, b, st, launch, grid_out);
}

hipError_t launch_reduce_records(const double *partials, int count, int width, double *out_dev,
                                 hipStream_t st) {
    if (count < 1 || count > kMaxReduceBlocks || width < 1 || width > kMaxReduceWidth)
        return hipErrorInvalidValue;
    reduce_records<<<1, kBlock, 0, st>>>(partials, count, width, out_dev);
    return hipGetLastError();
}

hipError_t launch_norm(const float2 *amp, int n, double *partials, double *out_dev,
                       hipStream_t st) {
    const int nb = reduce_blocks_for(n, 0);
    const uint64_t dim = uint64_t(1) << n;
    if (n <= 31)
        norm_partials<uint32_t><<<nb, kBlock, 0, st>>>(amp, uint32_t(dim), partials);
    else
        norm_partials<uint64_t><<<nb, kBlock, 0, st>>>(amp, dim, partials);
    reduce_records<<<1, kBlock, 0, st>>>(partials, nb, 1, out_dev);
    return hipGetLastError();
}

hipError_t launch_zweights(const float2 *amp, int n, double *partials, double *out_dev, hipStream_t st) {
    if (n < 1 || n > kZRecord - 1 || n - 8 > 11 + kZIterBits) return hipErrorInvalidValue;
    // chunks of at least 256 amplitudes, at most kMaxReduceBlocks of them
    const int lb = n - 8 < 11 ? (n - 8 > 0 ? n - 8 : 0) : 11;
    const int c = n - lb;
    const unsigned nb = 1u << lb;
    if (n <= 31) zweight_partials<uint32_t><<<nb, kBlock, 0, st>>>(amp, n, c, partials);
    else zweight_partials<uint64_t><<<nb, kBlock, 0, st>>>(amp, n, c, partials);
    reduce_records<<<1, kBlock, 0, st>>>(partials, int(nb), kZRecord, out_dev);
    return hipGetLastError();
}

hipError_t launch_rdm(const float2 *amp, int n, int k, const int *t_sorted, double *partials,
                      double *out_dev, hipStream_t st) {
    const int nb = reduce_blocks_for(n, k);
    TargetArgs ta;
    for (int b = 0; b < kMaxGateQubits; ++b) ta.t[b] = b < k ? t_sorted[b] : 0;
    const uint64_t groups = uint64_t(1) << (n - k);
    const int width = 2 << (2 * k);
    if (k == 1) {
        if (n <= 31) rdm_partials<1, uint32_t><<<nb, kBlock, 0, st>>>(amp, uint32_t(groups), ta, partials);
        else rdm_partials<1, uint64_t><<<nb, kBlock, 0, st>>>(amp, groups, ta, partials);
    } else if (k == 2) {
        if (n <= 31) rdm_partials<2, uint32_t><<<nb, kBlock, 0, st>>>(amp, uint32_t(groups), ta, partials);
        else rdm_partials<2, uint64_t><<<nb, kBlock, 0, st>>>(amp, groups, ta, partials);
    } else {
        return hipErrorInvalidValue;
    }
    reduce_records<<<1, kBlock, 0, st>>>(partials, nb, width, out_dev);
    return hipGetLastError();
}

hipError_t launch_apply_copy_norm(const float2 *in, float2 *out, int n, const GateDesc &g,
                                  double *partials, double *out_dev, hipStream_t st) {
    const int nb = reduce_blocks_for(n, g.k);
    const uint64_t groups = uint64_t(1) << (n - g.k);
    if (g.k == 1) {
        if (n <= 31) apply_copy_norm<1, uint32_t><<<nb, kBlock, 0, st>>>(in, out, uint32_t(groups), make_args<1>(g), partials);
        else apply_copy_norm<1, uint64_t><<<nb, kBlock, 0, st>>>(in, out, groups, make_args<1>(g), partials);
    } else if (g.k == 2) {
        if (n <= 31) apply_copy_norm<2, uint32_t><<<nb, kBlock, 0, st>>>(in, out, uint32_t(groups), make_args<2>(g), partials);
        else apply_copy_norm<2, uint64_t><<<nb, kBlock, 0, st>>>(in, out, groups, make_args<2>(g), partials);
    } else {
        return hipErrorInvalidValue;
    }
    reduce_records<<<1, kBlock, 0, st>>>(partials, nb, 2, out_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------- allocation-free sampling

// The sampling buffers of qs_sample_measurements_noalloc: a fixed array per
// GPU, held until the process ends (4.5 MiB: block sums and prefix for up to
// 2^28 amplitudes, the norm, up to 2^16 bitstrings).  Host code must not pass
// `scratch` itself to a kernel (in host code the name is a stand-in, not a
// device address): it uses the address noalloc_scratch looked up.
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_dev[64] = {};  // per device, filled once
}  // namespace

hipError_t noalloc_scratch(int device, double **out) {
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[device] = static_cast<double *>(p);
    }
    *out = g_scratch_dev[device];
    return hipSuccess;
}

hipError_t launch_sample(const float2 *amp, int n, double *sums, double *incl, uint64_t seed,
                         uint32_t traj, uint32_t circ, int n_samples, const ReadoutDesc &ro,
                         uint64_t *out_dev, double *norm_dev, hipStream_t st) {
    const int B = n < kSampleBlockBits ? n : kSampleBlockBits;
    const int64_t nb = int64_t(1) << (n - B);
    const int64_t n_tiles = (nb + kScanTile - 1) / kScanTile;
    if (n_tiles > kScanMaxTiles) return hipErrorInvalidValue;
    const unsigned sum_grid = unsigned((nb + kBlock / 64 - 1) / (kBlock / 64));
    if (n <= 31)
        sample_block_sums<uint32_t><<<sum_grid, kBlock, 0, st>>>(amp, B, nb, sums);
    else
        sample_block_sums<uint64_t><<<sum_grid, kBlock, 0, st>>>(amp, B, nb, sums);
    sample_scan_tiles<<<unsigned(n_tiles), kScanThreads, 0, st>>>(sums, nb, incl);
    // the block sums have been read: their first n_tiles slots take the offsets
    sample_scan_offsets<<<1, kScanThreads, 0, st>>>(incl, nb, int(n_tiles), sums, norm_dev);
    if (n_tiles > 1)
        sample_scan_add<<<unsigned((nb - kScanTile + kBlock - 1) / kBlock), kBlock, 0, st>>>(incl, nb, sums);
    if (n_samples > 0) {
        const unsigned grid = unsigned((n_samples + kBlock / 64 - 1) / (kBlock / 64));
        if (B == 10 && n <= 31)
            sample_draw<uint32_t, 16><<<grid, kBlock, 0, st>>>(amp, n, B, incl, nb, norm_dev, seed, traj,
                                                               circ, n_samples, ro, out_dev);
        else if (B == 10)
            sample_draw<uint64_t, 16><<<grid, kBlock, 0, st>>>(amp, n, B, incl, nb, norm_dev, seed, traj,
                                                               circ, n_samples, ro, out_dev);
        else
            sample_draw<uint32_t, 0><<<grid, kBlock, 0, st>>>(amp, n, B, incl, nb, norm_dev, seed, traj,
                                                              circ, n_samples, ro, out_dev);
    }
    return hipGetLastError();
}

}  // namespace qs
