/*
 * qs.h -- C ABI of the MI355X noisy quantum-trajectory state-vector library.
 *
 * Method: arXiv 2111.02396 (Isakov et al., "Simulations of Quantum Circuits
 * with Approximate Noise using qsim and Cirq").  Fused k-qubit gates are
 * applied to a complex64 state vector of 2^n amplitudes (Section 3.1,
 * Algorithm 1; fusion in Section 3.2) and one Kraus operator per channel is
 * sampled per trajectory with the delayed inner-product scheme (Section 3.5,
 * Algorithm 2) or, for comparison, the conventional scheme it replaces.
 *
 * Conventions shared by every call:
 *   - qubit q is bit q of an amplitude index (little-endian);
 *   - amplitudes are complex64, interleaved (re, im), contiguous, 8*2^n bytes;
 *   - a matrix acting on targets[0..k-1] is 2^k x 2^k, row-major, complex128
 *     interleaved (re, im), with row/column bit j belonging to targets[j];
 *     targets are distinct and in [0, n); 1 <= k <= 5; 1 <= n <= 34;
 *   - the state starts as |0...0>; matrices need not be unitary;
 *   - normalisation is lazy: the stored vector psi may have any positive norm
 *     N = <psi|psi>; Kraus probabilities and samples always use psi/sqrt(N);
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 *     (seed mod 2^32, seed >> 32) and counter (index, trajectory, circuit id,
 *     stream); stream 0 = channel draws (index = channel ordinal), 1 =
 *     measurement samples (index = sample), 2 = readout flips (index =
 *     sample * n + qubit); a draw is the top 53 bits of output words 1:0
 *     scaled by 2^-53, a double in [0, 1).
 *
 * Ownership: a state handle owns its device memory unless the caller lends a
 * buffer (e.g. a PyTorch tensor), which must outlive the handle.  Host input
 * arrays are read only during the call; every output is caller-allocated.
 *
 * Streams: work is enqueued on the handle's HIP stream; calls that return
 * host values synchronise that stream.  A handle is used by one host thread
 * at a time; distinct handles on distinct streams are independent.
 *
 * Errors: every call returns a qs_status.  Arguments are validated before any
 * work is enqueued, so QS_ERR_INVALID_ARGUMENT leaves the state untouched.
 * QS_ERR_DEVICE poisons the handle: every later call on it returns
 * QS_ERR_DEVICE until qs_destroy_state.  qs_last_error_message() describes
 * the most recent failure on the calling thread.
 */
#ifndef QS_H
#define QS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QS_OK = 0,
    QS_ERR_INVALID_ARGUMENT = -1,
    QS_ERR_OUT_OF_MEMORY = -2,
    QS_ERR_DEVICE = -3,
    QS_ERR_ZERO_NORM = -4,
    QS_ERR_NOT_SUPPORTED = -5
} qs_status;

/* Branch-selection scheme for channels (Section 3.5). */
typedef enum {
    QS_KRAUS_DELAYED = 0, /* Algorithm 2: lower bounds first, inner products only when r >= s */
    QS_KRAUS_NAIVE = 1,   /* conventional: apply K_i, take its norm, for i in order */
    QS_KRAUS_CONVENTIONAL_INPLACE = 2 /* conventional rule (r < p_i, i in order) with every p_i
                                         from one in-place read pass per channel and the chosen
                                         K_i folded into the next fused block: the conventional
                                         method without its scratch state */
} qs_kraus_mode;

typedef struct qs_state_s *qs_state;

enum { QS_OP_GATE = 0, QS_OP_CHANNEL = 1 };

/* One operation of a circuit (Section 2: a Circuit is Moments of Operations;
 * a channel is given by its Kraus operators). */
typedef struct {
    int32_t kind;       /* QS_OP_GATE or QS_OP_CHANNEL */
    int32_t k;          /* number of target qubits; gates 1..5, channels 1..2 */
    int32_t targets[5]; /* targets[0..k-1]; matrix bit j <-> targets[j] */
    int32_t n_mats;     /* 1 for a gate; the number of Kraus operators (1..16) for a channel */
    int64_t mat_offset; /* complex-element offset of the first matrix in mat_pool; a
                           channel's Kraus operators follow each other */
} qs_op;

/* A time-ordered circuit over n_qubits with its matrices in one pool. */
typedef struct {
    int32_t n_qubits;
    int32_t n_ops;
    const qs_op *ops;        /* host, n_ops entries */
    const double *mat_pool;  /* host, complex128 interleaved */
    int64_t pool_len;        /* complex elements in mat_pool */
} qs_circuit;

enum {
    QS_TRAJ_RETURN_STATE = 1u, /* copy the last trajectory's final amplitudes to final_state */
    QS_TRAJ_TIME_KERNELS = 2u, /* bracket every fused-gate launch with HIP events on the
                                  state's stream and report their summed durations */
    QS_TRAJ_NO_GRAPH = 4u,     /* launch every sweep directly (the default; overrides
                                  QS_TRAJ_GRAPH) */
    QS_TRAJ_GRAPH = 8u         /* replay the default plan's sweeps from a HIP graph where
                                  possible (see qs_run_trajectories) */
};

typedef struct {
    int64_t n_traj;        /* trajectories to run: indices traj_offset .. traj_offset+n_traj-1 */
    int64_t traj_offset;   /* first trajectory index (resume, or a shard of a larger run) */
    uint64_t seed;         /* Philox key */
    uint32_t circuit_id;   /* Philox counter word 2 */
    int32_t mode;          /* qs_kraus_mode */
    int32_t max_fuse;      /* largest fused gate (Section 3.2), 1..5; 0 = autotuned: the
                              delayed-mode driver times the circuit's default plan (every
                              channel at its most likely pick) on the device for each
                              candidate width (2..5 below 16 qubits, else 3..5) and keeps
                              the fastest, cached per circuit and state size for the life
                              of the process (the conventional modes use 4) */
    int32_t tile_bits;     /* LDS tile sweeps: fused gates whose qubits fit a tile of this
                              many index bits (bits 0..3 always included) share one pass
                              over the state; 0 = library default (13), or, when max_fuse
                              is 0, autotuned with it over 12..14; 1 = off (one pass per
                              fused gate), otherwise 10..14 */
    int32_t n_samples;     /* measurement samples per trajectory (>= 0) */
    const double *p0to1;   /* per-qubit readout P(read 1 | state 0), host, or NULL */
    const double *p1to0;   /* per-qubit readout P(read 0 | state 1), host, or NULL */
    uint32_t flags;        /* QS_TRAJ_* */
} qs_traj_params;

typedef struct {
    uint64_t *bitstrings;   /* host [n_traj * n_samples], or NULL */
    int8_t *kraus_choices;  /* host [n_traj * n_channels] chosen Kraus index, or NULL */
    int8_t *kraus_paths;    /* host [n_traj * n_channels]: 0 picked from the bounds,
                               1 picked after inner products, or NULL */
    int32_t *n_slow;        /* host [n_traj] channels that needed inner products, or NULL */
    void *final_state;      /* host complex64 [2^n] (QS_TRAJ_RETURN_STATE), or NULL */
    int64_t sweeps;         /* out: kernel passes over the state (gate blocks + reductions) */
    int64_t gate_sweeps;    /* out: fused-gate passes only */
    double host_seconds;    /* out: wall time of the call */
    double gate_kernel_ms;  /* out (QS_TRAJ_TIME_KERNELS): time during which the call's fused-gate
                               sweeps ran (HIP events bracketing each run of back-to-back
                               sweeps; with several streams, the union of their brackets) */
    int64_t gate_kernel_launches; /* out (QS_TRAJ_TIME_KERNELS): launches timed */
    int64_t gate_k_launches[6];   /* out: fused-gate launches by width k = 1..5 (index k) */
    int64_t zero_start_sweeps;    /* out: gate sweeps that began from |0...0> written on chip and
                                     read no state (one write of the state instead of a read and
                                     a write); counted among gate_sweeps */
    double *z_expect;             /* host [n_traj * n_qubits]: <Z_q> of each trajectory's final
                                     state (as qs_expectation_z), or NULL to skip the pass */
    int32_t max_fuse_used;        /* out: the fusion width the call ran with */
    int32_t tile_bits_used;       /* out: the tile width the call ran with (1 = no tiles) */
    double tune_ms;               /* out: wall time this call spent autotuning (0 on a cached
                                     or fixed choice) */
    int64_t graph_replays;        /* out: trajectories whose sweeps ran as a HIP-graph replay */
} qs_traj_result;

/* ---- state lifecycle ---------------------------------------------------- */

/* Create an n-qubit state set to |0...0> (Section 3: the simulator keeps the
 * 2^n complex amplitudes of the state, in single precision; Section 4.1: a
 * state takes 8 * 2^n bytes, up to twice that while a noisy trajectory needs
 * a second state, as the conventional method does here).
 * device_buf: NULL = the library allocates 8*2^n bytes; otherwise a device
 *   buffer of at least 8*2^n bytes (buf_bytes), 16-byte aligned (kernels move
 *   amplitude pairs), that the caller keeps alive.
 * hip_stream: the hipStream_t to enqueue on, or NULL for the null stream.
 * Errors: INVALID_ARGUMENT (n outside 1..34, short or misaligned buffer),
 * OUT_OF_MEMORY (allocation refused or free device memory below 8*2^n),
 * DEVICE. */
qs_status qs_create_state(int n_qubits, void *device_buf, size_t buf_bytes, void *hip_stream,
                          qs_state *out);

/* Release the handle, its device buffers and any pending operations. */
qs_status qs_destroy_state(qs_state s);

/* Reset to |0...0> and drop pending operations. */
qs_status qs_reset_state(qs_state s);

/* Device address of the amplitudes (pending operations are NOT flushed). */
qs_status qs_state_device_ptr(qs_state s, void **out);

/* Number of qubits of the state. */
qs_status qs_state_qubits(qs_state s, int *n_out);

/* Apply every deferred operation now (Algorithm 2, step 12). */
qs_status qs_flush(qs_state s);

/* Flush, then copy 8*2^n bytes of complex64 amplitudes to host memory (syncs). */
qs_status qs_copy_state_to_host(qs_state s, void *host_out, size_t bytes);

/* Replace the amplitudes with host complex64 data (8*2^n bytes; drops pending ops). */
qs_status qs_load_state_from_host(qs_state s, const void *host_in, size_t bytes);

/* Copy the amplitudes of `src` into `dst` on the device (one read and one
 * write of 8*2^n bytes, 16-byte accesses).  src's pending operations are
 * applied first; dst's are dropped.  The copy runs on dst's stream after the
 * work already enqueued on src's stream, and later work on src's stream waits
 * for it.  Both handles keep their own buffers (dst == src is a no-op).
 * Errors: INVALID_ARGUMENT (null handle, different qubit counts),
 * NOT_SUPPORTED (states on different devices), DEVICE. */
qs_status qs_copy_state(qs_state dst, qs_state src);

/* ---- the hot path ------------------------------------------------------- */

/* Apply one (already fused) k-qubit matrix to the state: Section 3.1,
 * Algorithm 1 -- for each of the 2^(n-k) index groups, gather the 2^k
 * amplitudes at the target bits, multiply by the matrix, scatter back.
 * Deferred operations are applied first.  matrix: host complex128 2^k x 2^k.
 * Errors: INVALID_ARGUMENT (k, targets, non-finite entries), DEVICE. */
qs_status qs_apply_fused_gate(qs_state s, int k, const int *targets, const double *matrix);

/* Sample and apply one Kraus operator of a channel (Section 3.5).
 * kraus: host, n_kraus consecutive complex128 2^k x 2^k matrices (k = 1..2,
 * n_kraus = 1..16) with sum K_i^dag K_i = I.  The draw is
 * r = U53(Philox(seed; channel_index, traj, 0, stream 0)).
 * QS_KRAUS_DELAYED (Algorithm 2): with bounds pbar_i = lambda_min(K_i^dag K_i),
 *   r < sum pbar_i picks from the bounds alone and defers K_i (returns
 *   without device work); otherwise the deferred operations are applied, one
 *   read pass forms the FP64 expectations <psi|K_i^dag K_i - pbar_i I|psi>/N
 *   in place (step 14), and the residual picks i; K_i/sqrt(p_i N) is deferred.
 * QS_KRAUS_NAIVE: for i in order, K_i psi is written to a scratch state (2x
 *   memory) with its FP64 norm in the same pass; r < p_i keeps it.
 * QS_KRAUS_CONVENTIONAL_INPLACE: the same rule, with p_i = <psi|K_i^dag K_i|psi>/N
 *   from one in-place read pass (Algorithm 2's second loop with every bound 0).
 * chosen_out (may be NULL) receives the chosen index; path_out (may be NULL)
 * receives 0 (picked from the bounds) or 1 (inner products were needed).
 * Errors: INVALID_ARGUMENT, NOT_SUPPORTED (k > 2), ZERO_NORM (the state or
 * every candidate has zero norm), DEVICE. */
qs_status qs_apply_channel(qs_state s, int k, const int *targets, int n_kraus,
                           const double *kraus, uint64_t seed, uint32_t traj,
                           uint32_t channel_index, qs_kraus_mode mode, int *chosen_out,
                           int *path_out);

/* N = <psi|psi> of the stored vector, accumulated in FP64 with a fixed
 * reduction order (bit-identical run to run).  Section 3.5 defines each
 * Kraus probability as p_i = <Psi|K_i^dag K_i|Psi> on the normalised state;
 * with lazy normalisation every probability and sample divides by this N.
 * Flushes; synchronises.  Errors: INVALID_ARGUMENT (null output), DEVICE. */
qs_status qs_norm(qs_state s, double *norm_sq_out);

/* Observable estimation on the trajectory's state (Section 3.5: an
 * expectation is averaged over trajectories, each taken on the normalised
 * state psi/sqrt(N)).
 * qs_expectation_z: z_out[q] = <psi|Z_q|psi>/N for every qubit q, from one
 * FP64 read pass (sums of |psi_x|^2 over the indices with bit q set; fixed
 * reduction order).  z_out: host double [n_qubits].
 * qs_expectation: <psi|O|psi>/N for a Hermitian O on k = 1..2 qubits,
 * given as a 2^k x 2^k complex128 row-major matrix whose row/column index
 * bit j is targets[j] (the convention of qs_apply_fused_gate), taken as
 * Tr(O R)/Tr(R) with R the FP64 reduced density matrix of the targets.
 * Both flush and synchronise.  Errors: INVALID_ARGUMENT (null pointer,
 * target out of range or repeated, O not Hermitian to 1e-12 relative),
 * NOT_SUPPORTED (k > 2), ZERO_NORM, DEVICE. */
qs_status qs_expectation_z(qs_state s, double *z_out);
qs_status qs_expectation(qs_state s, int k, const int *targets, const double *observable,
                         double *value_out);

/* Measure every qubit n_samples times (inverse CDF of |psi_x|^2/N in index
 * order: sample s takes the smallest x with u_s N < C(x), C the inclusive
 * prefix of |psi_x|^2; the last index if none), then flip bit q with
 * probability p0to1[q] or p1to0[q] by its true value (Section 5.1.2 readout
 * misidentification), using Philox streams 1 and 2 with circuit id 0.
 * bitstrings_out: host uint64 [n_samples].  Flushes; synchronises.
 * Errors: INVALID_ARGUMENT, ZERO_NORM, DEVICE. */
qs_status qs_sample_measurements(qs_state s, uint64_t seed, uint32_t traj, int n_samples,
                                 const double *p0to1, const double *p1to0,
                                 uint64_t *bitstrings_out);

/* For callers that cannot allocate device or pinned memory (tight serving
 * loops, harnesses that forbid hipMalloc, code that must not allocate while
 * other work is being captured): qs_sample_measurements with the
 * same arguments, the same kernels and bit-identical bitstrings, whose
 * device buffers (block sums, prefix, norm, bitstrings) live in one fixed
 * 4.5 MiB array per GPU that the library holds until the process ends.  It
 * calls no hipMalloc, hipHostMalloc or hipFree: the norm and the bitstrings
 * are copied straight into the caller's host memory.
 * Limits: the state has at most 28 qubits and 0 <= n_samples <= 65536;
 * beyond them it returns QS_ERR_INVALID_ARGUMENT without device work.  The
 * state must have no deferred operations (applying them may need staging
 * memory): call qs_flush first, else QS_ERR_INVALID_ARGUMENT.
 * Every call on one GPU uses that GPU's array, so calls that overlap on one
 * GPU (from several host threads or streams) race; the array keeps the last
 * call's contents, and every call writes all it reads.
 * Errors: INVALID_ARGUMENT, ZERO_NORM, DEVICE. */
qs_status qs_sample_measurements_noalloc(qs_state s, uint64_t seed, uint32_t traj, int n_samples,
                                         const double *p0to1, const double *p1to0,
                                         uint64_t *bitstrings_out);

/* Run n_traj noisy trajectories of one circuit on this state's buffer and
 * stream (Section 3.5): per trajectory, reset to |0...0>, draw one r per
 * channel, classify each channel as picked-from-bounds or needing inner
 * products (Algorithm 2, steps 1-11; state-independent), fuse the resulting
 * operator list into blocks of at most max_fuse qubits (Section 3.2) split
 * at the channels that need inner products, apply the blocks, resolve those
 * channels in place (steps 12-20), and finally sample.  QS_KRAUS_NAIVE
 * resolves every channel by the conventional method instead, and
 * QS_KRAUS_CONVENTIONAL_INPLACE by the conventional rule with in-place
 * inner products (every channel takes the inner-product path).
 * With QS_TRAJ_GRAPH, on small states (delayed mode, at most 22 qubits, two
 * or more trajectories, every sweep a tile sweep): the sweeps of the
 * circuit's default plan are captured once per call into a HIP graph whose
 * kernels read each fused block's matrix from a fixed device slot; a
 * trajectory whose channels are all picked from the bounds then writes its
 * patched blocks into their slots (one host-to-device copy on the stream)
 * and replays the graph, instead of launching the sweeps one by one.  The
 * results are those of the direct launches (the same kernels on the same
 * matrices).  Off by default: on MI355X with ROCm 7 the replays measured a
 * few percent slower than direct launches of the same sweeps.
 * The circuit's n_qubits must equal the state's.  Results are written to the
 * caller's host arrays in r.  On return the state holds the last trajectory's
 * final vector (lazily normalised; what QS_TRAJ_RETURN_STATE copies out), or
 * is unchanged when n_traj is 0.  Errors: INVALID_ARGUMENT, ZERO_NORM, DEVICE. */
qs_status qs_run_trajectories(qs_state s, const qs_circuit *c, const qs_traj_params *p,
                              qs_traj_result *r);

/* The trajectory range of p split over several states that run at once
 * (Section 3.5: trajectories are independent).  The range is cut into
 * n_states contiguous chunks (the first n_traj mod n_states chunks one
 * trajectory longer); chunk j runs as qs_run_trajectories on states[j], from
 * a host thread of its own, so the chunks' kernels overlap on the device
 * when the states use different streams (one sweep's load and store ramps
 * are then filled by another's work).  Every trajectory's draws depend only
 * on (seed, trajectory index, circuit id), so all outputs equal those of
 * one qs_run_trajectories call over the same range.  Results go to r's
 * arrays at each trajectory's position; final_state (QS_TRAJ_RETURN_STATE)
 * is the range's last trajectory; the counters are sums over the chunks
 * (gate_kernel_ms is the union over the streams: time during which at
 * least one of the call's sweeps was running).
 * states: 1..16 distinct handles, each with n_qubits equal to the
 * circuit's.  Errors: as qs_run_trajectories (the first failing chunk's). */
qs_status qs_run_trajectories_concurrent(qs_state *states, int n_states, const qs_circuit *c,
                                         const qs_traj_params *p, qs_traj_result *r);

/* ---- batched persistent launch ------------------------------------------ */

/* One circuit of a batched launch and where its results go. */
typedef struct {
    const qs_circuit *circuit; /* 1 <= n_qubits <= 18; every channel a mixture of unitaries
                                  (all K_i^dag K_i multiples of I, so Algorithm 2 never
                                  needs inner products) */
    int64_t n_traj;            /* trajectories traj_offset .. traj_offset+n_traj-1 */
    int64_t traj_offset;
    uint64_t seed;             /* Philox key */
    uint32_t circuit_id;       /* Philox counter word 2 */
    int32_t n_samples;         /* per trajectory, 0..4096 */
    const double *p0to1;       /* per-qubit readout P(1|0), host, or NULL */
    const double *p1to0;       /* per-qubit readout P(0|1), host, or NULL */
    uint64_t *bitstrings;      /* host out [n_traj * n_samples]; pinned host memory
                                  (hipHostMalloc) receives 16384 or more samples with one
                                  transfer and no staging copy */
    int8_t *kraus_choices;     /* host out [n_traj * n_channels], or NULL */
} qs_batch_item;

typedef struct {
    int32_t max_fuse;          /* 1..5; 0 = autotuned: each candidate width 2..5 runs the
                                  batch cut to two trajectories per circuit, timed whole
                                  (planning, upload, launch), the fastest is kept (cached
                                  per batch of circuits for the life of the process) */
    uint32_t flags;            /* QS_TRAJ_TIME_KERNELS: time the launch with HIP events */
    void *hip_stream;          /* hipStream_t, or NULL */
} qs_batch_params;

typedef struct {
    int64_t jobs;              /* trajectories run */
    int64_t resident_jobs;     /* of which kept their state in LDS throughout */
    int64_t gate_blocks;       /* fused blocks applied, summed over trajectories */
    double host_seconds;       /* wall time of the call */
    double plan_seconds;       /* host planning (draws, patched blocks, packing) */
    double kernel_ms;          /* QS_TRAJ_TIME_KERNELS: the persistent launch */
    int32_t max_fuse_used;     /* the fusion width the launch ran with */
    int32_t pad;
    double tune_ms;            /* wall time spent autotuning in this call (0 if cached/fixed) */
} qs_batch_result;

/* Many small noisy circuits in ONE persistent kernel launch (Section 3.5's
 * trajectories, run side by side).  Every trajectory's draws are resolved
 * from the Kraus bounds on the host (mixtures only), each circuit is fused
 * once (Section 3.2) and a trajectory carries only the blocks whose picks
 * differ from the circuit's most likely ones.  On the device each
 * workgroup takes trajectories in turn: a state of n <= 13 qubits lives in
 * LDS for the whole trajectory; a larger one streams 2^12-amplitude tiles
 * of a per-workgroup slot in device memory, one pass per tile sweep.  The
 * workgroup then samples with readout flips exactly as
 * qs_sample_measurements does (same Philox streams, circuit id from the
 * item).  Results are written to each item's host arrays.
 * Only mixtures of unitaries are taken: for them Algorithm 2 never needs an
 * inner product (the bounds sum to one), so every trajectory's program is
 * fixed before the launch and the workgroups never wait on a reduction.  A
 * channel with rank-deficient or non-normal Kraus operators (amplitude or
 * phase damping) needs the state-dependent second loop of Algorithm 2;
 * circuits with such channels go through qs_run_trajectories (the serving
 * loop sends them to its slot lane).
 * Errors: INVALID_ARGUMENT, NOT_SUPPORTED (n > 18, a channel that is not a
 * mixture), OUT_OF_MEMORY, DEVICE. */
qs_status qs_run_batched(const qs_batch_item *items, int n_items, const qs_batch_params *p,
                         qs_batch_result *r);

/* ---- host-side helpers (no device work) --------------------------------- */

/* Kraus lower bounds pbar_i = lambda_min(K_i^dag K_i), clamped at 0
 * (Section 3.5), and whether every K_i^dag K_i is a multiple of I (then the
 * bounds sum to one and the channel never needs inner products).
 * pbar_out: host double [n_kraus]; mixture_out: host int. */
qs_status qs_kraus_bounds(int k, int n_kraus, const double *kraus, double *pbar_out,
                          int *mixture_out);

/* Gate fusion (Section 3.2) of a channel-free circuit into blocks of at most
 * max_fuse qubits (gates wider than max_fuse form their own block).
 * Outputs (capacity n_ops blocks): n_blocks_out; block_k[b]; block_targets
 * [5*b..] ascending; block_mats[b] = 32*32 complex128 slots (only the
 * leading 2^k x 2^k used, row-major); op_block[o] = block of op o.  Applying
 * the blocks in order equals applying the gates in time order. */
qs_status qs_fusion_plan(const qs_circuit *c, int max_fuse, int32_t *n_blocks_out,
                         int32_t *block_k, int32_t *block_targets, double *block_mats,
                         int32_t *op_block);

/* Tile-sweep grouping of the blocks of qs_fusion_plan (same max_fuse): the
 * order in which the trajectory driver applies them, one pass over the state
 * per sweep.  Outputs (capacity n_ops): n_sweeps_out; order_out[i] = block
 * applied i-th; sweep_of_order[i] = its sweep; sweep_bits[s] = bit mask of
 * the index bits staged in LDS by sweep s (bits 0..3 always included).
 * tile_bits as in qs_traj_params (0 = 13).  Host only. */
qs_status qs_sweep_plan(const qs_circuit *c, int max_fuse, int tile_bits, int32_t *n_sweeps_out,
                        int32_t *order_out, int32_t *sweep_of_order, uint64_t *sweep_bits);

/* Philox4x32-10 of one counter/key (the library's own generator). */
qs_status qs_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Description of the most recent failure on the calling thread ("" if none). */
const char *qs_last_error_message(void);

/* Library version string. */
const char *qs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QS_H */
