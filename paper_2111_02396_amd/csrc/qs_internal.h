// Internal interface between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qs {

constexpr int kMaxGateQubits = 5;
constexpr int kMaxChannelQubits = 2;
constexpr int kMaxQubits = 34;

// Threads per workgroup of the streaming kernels (four wave64 wavefronts).
constexpr int kBlock = 256;

// Reduction partial buffers hold at most this many workgroups' results.
constexpr int kMaxReduceBlocks = 2048;
// Widest per-workgroup reduction record: the 4x4 complex two-qubit
// reduced density matrix (32 doubles) plus two scalars.
constexpr int kMaxReduceWidth = 36;
// Z-expectation record: N, then sum |psi_x|^2 over x with bit q set, q < 34
constexpr int kZRecord = 35;

// Sampling blocks hold 2^kSampleBlockBits amplitudes.
constexpr int kSampleBlockBits = 10;

// A fused gate as the kernels see it: targets ascending, matrix rows and
// columns in that ascending-target bit order, complex64.
struct GateDesc {
    int k;
    int t[kMaxGateQubits];
    float2 m[32 * 32];  // leading (2^k)^2 entries used, row-major
};

struct TargetArgs {
    int t[kMaxGateQubits];
};

// Tiled sweeps: a tile is 2^tb amplitudes whose index bits are pos[0..tb-1]
// (ascending, always starting with bits 0..kTileLowBits-1); the gates g[0..n_gates-1]
// act in order on tile-local bit positions lt[] (ascending), with their
// matrices (2^k x 2^k complex64, rows/columns in lt order) read from device
// address `mat` (16-byte aligned) and, for k >= 3, staged in LDS at float2
// offset `lofs` (even) of a region of mat_total entries.
constexpr int kMaxTileBits = 14;
// Index bits every tile holds: a work-item moves an amplitude pair (bit 0)
// and eight consecutive lanes cover bits 1..3, so each group of eight lanes
// reads or writes one whole 128-byte line wherever the tile's other bits
// lie.  Requiring only these four (rather than a 512-byte row) leaves nine
// of a 13-bit tile's bits to the sweep's gates.
constexpr int kTileLowBits = 4;
constexpr int kDefaultTileBits = 13;  // tile sweeps when the caller asks for the default
constexpr int kMaxTileGates = 28;  // keeps TileArgs (a kernel argument) under 4 KiB
constexpr int kTileMinQubits = 10;
constexpr int kTileMatBudget = 4096;  // float2 of matrices staged per launch (32 KiB)
// What the sweep planner lets one launch stage: 13-bit tiles run two
// 512-work-item groups per CU, which fit the 160 KiB of LDS only with at
// most 16 KiB of matrices each (64 KiB tile + 16 KiB, twice).
inline int tile_mat_budget(int tile_bits) { return tile_bits == 13 ? 2048 : kTileMatBudget; }

// LDS float2 slots a gate's matrix takes in a tile launch: none for k <= 2
// (read from global memory), MFMA fragments for k = 3 (256 floats), k = 4
// (768 floats: three real 16x16 matrices) and k = 5 (3072 floats: three real
// 32x32 matrices; narrow tiles use the first 1024 slots for the plain
// matrix), each followed by a 64-entry per-lane offset table (32 slots).
__host__ __device__ inline int tile_mat_slots(int k) {
    return k <= 2 ? 0 : (k == 3 ? 160 : (k == 4 ? 416 : 1568));
}

struct TileGate {
    int k;
    int lt[kMaxGateQubits];
    int lofs;
    int pad;
    const float2 *mat;
    int tab[kMaxTileBits];  // LDS byte offset per logical bit, filled by launch_apply_tile
};

struct TileArgs {
    int tb;
    int pos[kMaxTileBits];
    int n_gates;
    int mat_total;
    int init_zero;  // 1: start from |0...0> written in LDS instead of reading the state
    // With rdm_out set, the launch also forms the reduced density matrix of
    // the qubit at tile-local bit rdm_lt on the state it leaves (Section 3.5's
    // inner products, from the tile in LDS after its gates): one record of
    // 8 doubles per workgroup, R[j][l] = sum v_j conj(v_l) as re, im in row
    // order, to be summed over the launch's workgroups.  Not with 5-qubit
    // blocks.
    int rdm_lt;
    double *rdm_out;
    TileGate g[kMaxTileGates];
};

// ---- batched persistent launch -------------------------------------------
// Device program of many small circuits, run one trajectory per workgroup
// iteration.  A circuit whose state fits in LDS (n <= kBatchLdsQubits) keeps
// it there for the whole trajectory; larger ones stream tiles of a per-
// workgroup global slot, one pass per sweep.
constexpr int kBatchLdsQubits = 13;
constexpr int kBatchMaxQubits = 18;
constexpr int kBatchTileBits = 12;
constexpr int kBatchMaxSamples = 4096;

struct BatchGate {
    int k;
    int lt[kMaxGateQubits];  // ascending; global bits (resident) or tile-local bits
    int mat;                 // float2 offset of the default matrix in the pool
    int m0, m1;              // the block's operations in the member table
};

struct BatchSweep {
    int tb;                  // tile bits (tiled circuits); n for resident ones
    int pos[kMaxTileBits];
    int g0, g1;              // gate range
};

struct BatchCircuit {
    int n;
    int resident;
    int s0, s1;              // sweep range
    int n_samples;
    int readout;             // offset of 2n doubles (e0[], e1[]) in the readout pool, or -1
    int g0, n_gates;         // the circuit's blocks (absolute first, count)
    int ch0, nch;            // the circuit's channels in the channel table
    int pool0, pool_len;     // float2 range of the circuit's default matrices in the pool
};

// A channel of a batched circuit (Algorithm 2's fast path for mixtures of
// unitaries: the pick is decided by r against the running sums of the
// fixed probabilities).
struct BatchChannel {
    int32_t nk;              // Kraus operators
    int32_t default_pick;    // the pick folded into the default block matrices
    int32_t pbar;            // offset of the nk probabilities in the pbar pool
    int32_t gate;            // block holding the channel, relative to the circuit's first
    int32_t unit;            // double2 offset of K_i / sqrt(pbar_i), i < nk, in the FP64 pool
    uint32_t identity;       // bit i: K_i is a multiple of I (left out of the fused product)
};

// One operation of a fused block, in the block's order, for recomputing the
// block's matrix when a trajectory's picks differ from the defaults.
struct BatchMember {
    int k;                   // qubits of the operation
    int lp[kMaxGateQubits];  // positions of its qubits (its own order) in the block's qubit list
    int src;                 // >= 0: double2 offset of a gate matrix in the FP64 pool;
                             // < 0: channel -src - 1 of the circuit
};

struct BatchJob {
    int circuit;
    uint32_t traj;           // Philox counter word 1
    uint32_t circ_id;        // Philox counter word 2
    int pad;
    uint64_t seed;           // Philox key
    int64_t out;             // first output sample
    int64_t choices;         // first recorded pick, or -1
};

struct BatchArgs {
    const BatchCircuit *circs;
    const BatchSweep *sweeps;
    const BatchGate *gates;
    const BatchJob *jobs;
    const float2 *mats;      // default block matrices
    const double *readout;
    const BatchChannel *chans;
    const double *pbar;
    const BatchMember *members;
    const double2 *fmats;    // FP64 gate and channel matrices for the members
    float2 *patched;         // per-workgroup matrices of the blocks a job's picks change
    int64_t patched_stride;  // float2 entries per workgroup
    int8_t *choices;         // recorded picks
    float2 *slots;           // per-workgroup state slots (tiled circuits)
    int64_t slot_amps;
    uint64_t *out;
    int n_jobs;
};

// Blocks per batched circuit: the job's patched-block flags are one bit each
// in a 2 KiB LDS array.
constexpr int kBatchMaxBlocks = 16384;

struct ReadoutDesc {
    int enabled;
    double e0[kMaxQubits];  // P(read 1 | 0)
    double e1[kMaxQubits];  // P(read 0 | 1)
};

// All launchers enqueue on `st` and return the launch status.

hipError_t launch_set_basis(float2 *amp, int n, uint64_t index, hipStream_t st);

hipError_t launch_scale(float2 *amp, int n, float s, hipStream_t st);

// dst[i] = src[i] for the 2^n amplitudes (16-byte accesses, grid-stride).
hipError_t launch_copy_state(float2 *dst, const float2 *src, int n, hipStream_t st);

// Algorithm 1 for one fused gate.  mat_dev: device copy of g.m
// ((2^k)^2 complex64, ascending-target order).  Gates with a target below 6
// go through the tiled path, the others through the direct path.
hipError_t launch_apply_gate(float2 *amp, int n, const GateDesc &g, const float2 *mat_dev,
                             hipStream_t st);

// Several gates in one sweep: every gate's targets are bits of the tile.
// grid_out (optional): the launch's workgroup count (its RDM record count).
hipError_t launch_apply_tile(float2 *amp, int n, const TileArgs &a, hipStream_t st,
                             int *grid_out = nullptr);
// Validates a and sets up its kernel instantiation without enqueueing
// anything (before a launch under stream capture).
hipError_t prepare_apply_tile(int n, const TileArgs &a);
hipError_t launch_apply_tile_impl(float2 *amp, int n, const TileArgs &a, hipStream_t st, bool launch,
                                  int *grid_out = nullptr);
// Sums `count` records of `width` doubles in index order into out_dev.
hipError_t launch_reduce_records(const double *partials, int count, int width, double *out_dev,
                                 hipStream_t st);

// FP64 reductions with a fixed tree.  Each writes `width` doubles to out_dev.
// norm: width 1 (sum |psi|^2).
hipError_t launch_norm(const float2 *amp, int n, double *partials, double *out_dev,
                       hipStream_t st);

// Per-qubit weights of the state in one read pass: out_dev[0] = N =
// sum |psi_x|^2, out_dev[1 + q] = sum over x with bit q set (FP64, fixed
// reduction order); <Z_q> = (N - 2 out[1 + q]) / N.  Width kZRecord.
hipError_t launch_zweights(const float2 *amp, int n, double *partials, double *out_dev,
                           hipStream_t st);

// Reduced density matrix R = sum_groups v v^dag over k <= 2 ascending
// targets: width 2*4^k doubles, R[j][l] at (2*(j*D+l), +1).
hipError_t launch_rdm(const float2 *amp, int n, int k, const int *t_sorted, double *partials,
                      double *out_dev, hipStream_t st);

// Conventional-method trial: out = M in (k <= 2), with sum |out|^2 and
// sum |in|^2 in one pass: width 2.
hipError_t launch_apply_copy_norm(const float2 *in, float2 *out, int n, const GateDesc &g,
                                  double *partials, double *out_dev, hipStream_t st);

int reduce_blocks_for(int n, int k);

// Sampling: block sums, a single-workgroup scan, then one thread per sample.
// sums / incl: device doubles [2^(n - B)] with B = min(n, kSampleBlockBits).
hipError_t launch_sample(const float2 *amp, int n, double *sums, double *incl,
                         uint64_t seed, uint32_t traj, uint32_t circ, int n_samples,
                         const ReadoutDesc &ro, uint64_t *out_dev, double *norm_dev,
                         hipStream_t st);

// Allocation-free sampling (qs_sample_measurements_noalloc): one fixed
// device array per GPU holds the block sums, their prefix, the norm and the
// bitstrings of one call.  Layout in doubles: sums [0, NB), incl [NB, 2 NB),
// norm at 2 NB, bitstrings (uint64) from 2 NB + 32 on.
constexpr int kNoAllocMaxQubits = 28;
constexpr int kNoAllocMaxSamples = 1 << 16;
constexpr size_t kNoAllocBlocks = size_t(1) << (kNoAllocMaxQubits - kSampleBlockBits);
constexpr size_t kNoAllocNormOffset = 2 * kNoAllocBlocks;
constexpr size_t kNoAllocOutOffset = 2 * kNoAllocBlocks + 32;
constexpr size_t kNoAllocDoubles = kNoAllocOutOffset + size_t(kNoAllocMaxSamples);

// Device address of that array on `device` (looked up once per device, with
// the device current; the caller's current device is restored).
hipError_t noalloc_scratch(int device, double **out);

// Device-side branch selection for a channel that needs inner products
// (Algorithm 2, steps 13-20): from the FP64 reduced density matrix R (as
// written by launch_rdm), e_i = Re Tr((K_i^dag K_i - pbar_i I) R) / N; the
// residual picks i (falling back to the last i with e_i > 0); then
// dst = cand[i] / sqrt((pbar_i + e_i) N) in complex64, where cand[i] is the
// fused block matrix with K_i in the channel's place.  Writes the pick to
// *choice; sets *err on a zero norm or weight.
struct SelectArgs {
    const double *rdm;     // 2 * D * D
    const double *excess;  // nk * D * D complex128, ascending target order
    const double *pbar;    // nk
    const double *cand;    // nk * Db * Db complex128
    float2 *dst;           // Db * Db
    int *choice;
    int *err;
    double resid;
    int nk, D, Db;
};

hipError_t launch_select(const SelectArgs &a, hipStream_t st);

// One persistent launch over all jobs; `grid` workgroups, each owning slot
// blockIdx.x of `slots` when it runs a tiled circuit.
hipError_t launch_batched(const BatchArgs &a, int grid, hipStream_t st);

// Workgroups the batched launch uses (persistent grid size).
int batched_grid();

}  // namespace qs
