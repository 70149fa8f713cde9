/*
 * Plain CPU oracle for the noisy quantum-trajectory state-vector method of
 * arXiv 2111.02396 (Isakov et al., "Simulations of Quantum Circuits with
 * Approximate Noise using qsim and Cirq").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the HIP path.  It is deliberately slow and literal: complex128,
 * single thread, no fusion, no deferral, no blocking, every operation
 * applied as the paper states it.
 *
 * Conventions: qubit q is bit q of an amplitude index; a matrix acting on
 * targets t[0..k-1] has row/column bit j on qubit t[j]; matrices are
 * row-major complex128 (interleaved re, im).
 *
 * Kraus lower bounds pbar_i (Section 3.5: the smallest squared singular
 * value of K_i) are computed by the Python side of the oracle with a
 * library eigenvalue routine and passed in.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------
 * Counter-based random numbers: Philox4x32 with 10 rounds, from the
 * published description (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11).  Each round multiplies counter
 * words 0 and 2 by two fixed 32-bit constants, keeps the high and low
 * halves of the 64-bit products, and mixes the high halves with the other
 * counter words and the round key; the key advances by two Weyl constants
 * between rounds.
 * ------------------------------------------------------------------------ */
#define OR_PHILOX_M0 0xD2511F53u
#define OR_PHILOX_M1 0xCD9E8D57u
#define OR_PHILOX_W0 0x9E3779B9u
#define OR_PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += OR_PHILOX_W0;
            k1 += OR_PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)OR_PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)OR_PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform double in [0, 1) from the top 53 of the 64 bits (w1:w0). */
double or_u53(uint32_t w0, uint32_t w1)
{
    uint64_t v = ((uint64_t)w1 << 32) | (uint64_t)w0;
    return (double)(v >> 11) * (1.0 / 9007199254740992.0);
}

/* One draw: key = (seed low, seed high), counter = (index, traj, circ, stream).
 * Streams: 0 channel draws, 1 measurement samples, 2 readout flips. */
double or_draw(uint64_t seed, uint32_t index, uint32_t traj, uint32_t circ, uint32_t stream)
{
    uint32_t ctr[4] = {index, traj, circ, stream};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    or_philox4x32_10(ctr, key, out);
    return or_u53(out[0], out[1]);
}

/* ------------------------------------------------------------------------
 * Gate application: Section 3.1, Algorithm 1.  For each of the 2^(n-k)
 * index groups, gather the 2^k amplitudes selected by the target bits,
 * multiply by the 2^k x 2^k matrix, scatter back.
 * ------------------------------------------------------------------------ */

/* Index of group i with zero bits inserted at the (ascending) target positions. */
static uint64_t group_base(uint64_t i, int k, const int *sorted_t)
{
    uint64_t x = i;
    for (int b = 0; b < k; ++b) {
        int t = sorted_t[b];
        uint64_t low = x & ((1ull << t) - 1ull);
        x = ((x >> t) << (t + 1)) | low;
    }
    return x;
}

static void sort_targets(int k, const int *t, int *sorted_t)
{
    for (int i = 0; i < k; ++i) sorted_t[i] = t[i];
    for (int i = 1; i < k; ++i)
        for (int j = i; j > 0 && sorted_t[j - 1] > sorted_t[j]; --j) {
            int tmp = sorted_t[j]; sorted_t[j] = sorted_t[j - 1]; sorted_t[j - 1] = tmp;
        }
}

/* Offset of local index j (bit b of j on qubit t[b]). */
static uint64_t local_offset(uint32_t j, int k, const int *t)
{
    uint64_t off = 0;
    for (int b = 0; b < k; ++b)
        if ((j >> b) & 1u) off |= 1ull << t[b];
    return off;
}

void or_apply_matrix(double *psi_ri, int n, int k, const int *t, const double *mat_ri)
{
    cplx *psi = (cplx *)psi_ri;
    const cplx *U = (const cplx *)mat_ri;
    int st[8];
    sort_targets(k, t, st);
    const uint32_t d = 1u << k;
    uint64_t off[32];
    for (uint32_t j = 0; j < d; ++j) off[j] = local_offset(j, k, t);
    const uint64_t groups = 1ull << (n - k);
    cplx v[32], w[32];
    for (uint64_t i = 0; i < groups; ++i) {
        uint64_t base = group_base(i, k, st);
        for (uint32_t j = 0; j < d; ++j) v[j] = psi[base + off[j]];
        for (uint32_t j = 0; j < d; ++j) {
            cplx s = 0.0;
            for (uint32_t l = 0; l < d; ++l) s += U[j * d + l] * v[l];
            w[j] = s;
        }
        for (uint32_t j = 0; j < d; ++j) psi[base + off[j]] = w[j];
    }
}

/* <psi|psi>, summed sequentially in index order. */
double or_norm_sq(const double *psi_ri, int n)
{
    const cplx *psi = (const cplx *)psi_ri;
    const uint64_t dim = 1ull << n;
    double s = 0.0;
    for (uint64_t x = 0; x < dim; ++x) {
        double re = creal(psi[x]), im = cimag(psi[x]);
        s += re * re + im * im;
    }
    return s;
}

static void scale_state(cplx *psi, int n, double f)
{
    const uint64_t dim = 1ull << n;
    for (uint64_t x = 0; x < dim; ++x) psi[x] *= f;
}

/* <psi| M |psi> for a 2^k x 2^k matrix M on targets t (no normalisation).
 * Section 3.5: the expectation in step 14 of Algorithm 2 is formed in place. */
void or_expectation(const double *psi_ri, int n, int k, const int *t, const double *mat_ri,
                    double *out_re, double *out_im)
{
    const cplx *psi = (const cplx *)psi_ri;
    const cplx *M = (const cplx *)mat_ri;
    int st[8];
    sort_targets(k, t, st);
    const uint32_t d = 1u << k;
    uint64_t off[32];
    for (uint32_t j = 0; j < d; ++j) off[j] = local_offset(j, k, t);
    const uint64_t groups = 1ull << (n - k);
    cplx acc = 0.0;
    cplx v[32];
    for (uint64_t i = 0; i < groups; ++i) {
        uint64_t base = group_base(i, k, st);
        for (uint32_t j = 0; j < d; ++j) v[j] = psi[base + off[j]];
        for (uint32_t j = 0; j < d; ++j) {
            cplx mv = 0.0;
            for (uint32_t l = 0; l < d; ++l) mv += M[j * d + l] * v[l];
            acc += conj(v[j]) * mv;
        }
    }
    *out_re = creal(acc);
    *out_im = cimag(acc);
}

/* E = K^dag K - c I (the "excess" matrix), complex128 d x d. */
static void excess_matrix(int d, const cplx *K, double c, cplx *E)
{
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            cplx s = 0.0;
            for (int m = 0; m < d; ++m) s += conj(K[m * d + a]) * K[m * d + b];
            E[a * d + b] = s - (a == b ? c : 0.0);
        }
}

/* ------------------------------------------------------------------------
 * Kraus-branch selection for one channel.
 *
 * Delayed inner product (Section 3.5, Algorithm 2):
 *   fast loop over i: if r < pbar_i pick i (no inner product); else r -= pbar_i.
 *   If every K_i is proportional to a unitary the bounds sum to one and a
 *   fall-through can only come from rounding: pick the last i with
 *   pbar_i > 0 on the fast path.
 *   Slow loop over i: e_i = <psi|(K_i^dag K_i - pbar_i I)|psi>/<psi|psi>
 *   (= p_i - pbar_i, formed without cancellation); if r < e_i pick i,
 *   else r -= e_i.  Rounding fall-through: the last i with e_i > 0.
 *
 * Conventional method (Section 3.5): for i in order, p_i = ||K_i psi||^2
 * (state normalised) by applying K_i to a copy; if r < p_i pick i, else
 * r -= p_i.  Rounding fall-through: the last i with p_i > 0.
 *
 * path: 0 = fast (no inner product), 1 = slow / conventional.
 * margin_fast / margin_slow: smallest |residual - threshold| over the
 * comparisons made in each loop (+inf when the loop did not run).
 * ------------------------------------------------------------------------ */
int or_select_branch(const double *psi_ri, int n, int k, const int *t, int n_kraus,
                     const double *kraus_ri, const double *pbar, int mixture, int mode,
                     double r, int *path, double *margin_fast, double *margin_slow)
{
    const cplx *K = (const cplx *)kraus_ri;
    const int d = 1 << k;
    double mf = INFINITY, ms = INFINITY;
    int choice = -1;
    const uint64_t dim = 1ull << n;
    if (mode == 0) {
        for (int i = 0; i < n_kraus; ++i) {
            double dist = fabs(r - pbar[i]);
            if (dist < mf) mf = dist;
            if (r < pbar[i]) { choice = i; break; }
            r -= pbar[i];
        }
        if (choice < 0 && mixture) {
            for (int i = n_kraus - 1; i >= 0; --i)
                if (pbar[i] > 0.0) { choice = i; break; }
        }
        if (choice >= 0) {
            *path = 0; *margin_fast = mf; *margin_slow = ms;
            return choice;
        }
        *path = 1;
        double N = or_norm_sq(psi_ri, n);
        cplx *E = (cplx *)malloc(sizeof(cplx) * d * d);
        int last_pos = -1;
        for (int i = 0; i < n_kraus; ++i) {
            excess_matrix(d, K + (size_t)i * d * d, pbar[i], E);
            double er, ei;
            or_expectation(psi_ri, n, k, t, (const double *)E, &er, &ei);
            double e = er / N;
            if (e > 0.0) last_pos = i;
            double dist = fabs(r - e);
            if (dist < ms) ms = dist;
            if (r < e) { choice = i; break; }
            r -= e;
        }
        free(E);
        if (choice < 0) choice = last_pos >= 0 ? last_pos : n_kraus - 1;
    } else {
        *path = 1;
        double N = or_norm_sq(psi_ri, n);
        cplx *phi = (cplx *)malloc(sizeof(cplx) * dim);
        int last_pos = -1;
        for (int i = 0; i < n_kraus; ++i) {
            memcpy(phi, psi_ri, sizeof(cplx) * dim);
            or_apply_matrix((double *)phi, n, k, t, (const double *)(K + (size_t)i * d * d));
            double p = or_norm_sq((const double *)phi, n) / N;
            if (p > 0.0) last_pos = i;
            double dist = fabs(r - p);
            if (dist < ms) ms = dist;
            if (r < p) { choice = i; break; }
            r -= p;
        }
        free(phi);
        if (choice < 0) choice = last_pos >= 0 ? last_pos : n_kraus - 1;
    }
    *margin_fast = mf;
    *margin_slow = ms;
    return choice;
}

/* Select for many r values on one fixed state (partition checks). */
void or_select_many(const double *psi_ri, int n, int k, const int *t, int n_kraus,
                    const double *kraus_ri, const double *pbar, int mixture, int mode,
                    int64_t n_r, const double *rs, int8_t *choices)
{
    for (int64_t m = 0; m < n_r; ++m) {
        int path;
        double mf, ms;
        choices[m] = (int8_t)or_select_branch(psi_ri, n, k, t, n_kraus, kraus_ri, pbar,
                                              mixture, mode, rs[m], &path, &mf, &ms);
    }
}

/* Apply the chosen Kraus operator and renormalise: psi <- K psi / ||K psi||. */
int or_apply_kraus_normalised(double *psi_ri, int n, int k, const int *t, const double *K_ri)
{
    or_apply_matrix(psi_ri, n, k, t, K_ri);
    double N = or_norm_sq(psi_ri, n);
    if (!(N > 0.0)) return -1;
    scale_state((cplx *)psi_ri, n, 1.0 / sqrt(N));
    return 0;
}

/* ------------------------------------------------------------------------
 * Measurement sampling (the paper measures every qubit at the end and
 * gives no sampling algorithm; this is inverse-CDF sampling in index
 * order).  N = sum |psi_x|^2 sequentially, C(x) = inclusive prefix.
 * Sample s: u = draw(stream 1, index s); x = min{x : u N < C(x)}, or the
 * last index if none.  Readout misidentification (Section 5.1.2): bit q
 * with true value b flips when draw(stream 2, index s*n + q) < e_b[q].
 * margin: min(uN - C(x-1), C(x) - uN) / N.
 * ------------------------------------------------------------------------ */
int or_sample(const double *psi_ri, int n, uint64_t seed, uint32_t traj, uint32_t circ,
              int64_t n_samples, const double *e0, const double *e1, uint64_t *out,
              double *margins)
{
    const cplx *psi = (const cplx *)psi_ri;
    const uint64_t dim = 1ull << n;
    double *C = (double *)malloc(sizeof(double) * dim);
    if (!C) return -1;
    double acc = 0.0;
    for (uint64_t x = 0; x < dim; ++x) {
        double re = creal(psi[x]), im = cimag(psi[x]);
        acc += re * re + im * im;
        C[x] = acc;
    }
    const double N = acc;
    for (int64_t s = 0; s < n_samples; ++s) {
        double u = or_draw(seed, (uint32_t)s, traj, circ, 1);
        double target = u * N;
        /* smallest x with target < C[x] */
        uint64_t lo = 0, hi = dim; /* answer in [lo, hi) ; hi == dim means none */
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (target < C[mid]) hi = mid; else lo = mid + 1;
        }
        uint64_t x = lo < dim ? lo : dim - 1;
        if (margins) {
            double below = x > 0 ? target - C[x - 1] : target;
            double above = C[x] - target;
            double m = below < above ? below : above;
            margins[s] = (N > 0.0) ? fabs(m) / N : 0.0;
        }
        if (e0 && e1) {
            for (int q = 0; q < n; ++q) {
                int b = (int)((x >> q) & 1ull);
                double v = or_draw(seed, (uint32_t)((uint64_t)s * (uint64_t)n + (uint64_t)q),
                                   traj, circ, 2);
                double e = b ? e1[q] : e0[q];
                if (v < e) x ^= 1ull << q;
            }
        }
        out[s] = x;
    }
    free(C);
    return 0;
}

/* ------------------------------------------------------------------------
 * One full trajectory over a time-ordered op list, starting from |0...0>.
 *
 * Op o: kinds[o] (0 gate, 1 channel), ks[o], targets[5*o .. 5*o+k-1],
 * n_mats[o] matrices starting at matrix ordinal first_mat[o]; matrix m
 * sits at complex offset mat_off[m] of mat_pool and has bound pbar[m].
 * mixture[o] != 0 marks a channel whose K_i^dag K_i are all multiples of I.
 *
 * Channel j (its ordinal among channels) draws r = draw(stream 0, index j).
 * Every channel consumes exactly one draw in both modes.
 * The state is renormalised after every channel (the stored vector stays a
 * unit vector), so the result is the normalised trajectory state.
 *
 * Outputs (per channel ordinal): choice, path, margins; samples and their
 * margins; the final state when psi_out != NULL (2 * 2^n doubles).
 * Returns 0, or -1 on a zero-norm state.
 * ------------------------------------------------------------------------ */
int or_run_trajectory(int n, int n_ops, const int32_t *kinds, const int32_t *ks,
                      const int32_t *targets, const int32_t *n_mats, const int64_t *first_mat,
                      const int64_t *mat_off, const double *mat_pool, const double *pbar,
                      const int32_t *mixture, int mode, uint64_t seed, uint32_t traj,
                      uint32_t circ, int64_t n_samples, const double *e0, const double *e1,
                      int8_t *choices, int8_t *paths, double *margin_fast, double *margin_slow,
                      uint64_t *samples, double *sample_margins, double *psi_out)
{
    const uint64_t dim = 1ull << n;
    cplx *psi = (cplx *)calloc(dim, sizeof(cplx));
    if (!psi) return -2;
    psi[0] = 1.0;
    uint32_t ch = 0;
    int rc = 0;
    for (int o = 0; o < n_ops; ++o) {
        int k = ks[o];
        int t[5];
        for (int b = 0; b < k; ++b) t[b] = targets[5 * o + b];
        const cplx *pool = (const cplx *)mat_pool;
        if (kinds[o] == 0) {
            or_apply_matrix((double *)psi, n, k, t, (const double *)(pool + mat_off[first_mat[o]]));
            continue;
        }
        /* channel */
        int nk = n_mats[o];
        int64_t m0 = first_mat[o];
        int d = 1 << k;
        /* the Kraus matrices of one channel are stored contiguously */
        const double *kraus = (const double *)(pool + mat_off[m0]);
        double r = or_draw(seed, ch, traj, circ, 0);
        int path;
        double mf, ms;
        double Nb = or_norm_sq((const double *)psi, n);
        if (!(Nb > 0.0)) { rc = -1; break; }
        scale_state(psi, n, 1.0 / sqrt(Nb));
        int c = or_select_branch((const double *)psi, n, k, t, nk, kraus, pbar + m0,
                                 mixture[o], mode, r, &path, &mf, &ms);
        if (choices) choices[ch] = (int8_t)c;
        if (paths) paths[ch] = (int8_t)path;
        if (margin_fast) margin_fast[ch] = mf;
        if (margin_slow) margin_slow[ch] = ms;
        if (or_apply_kraus_normalised((double *)psi, n, k, t,
                                      (const double *)((const cplx *)kraus + (size_t)c * d * d)) != 0) {
            rc = -1;
            break;
        }
        ++ch;
    }
    if (rc == 0 && n_samples > 0 && samples)
        rc = or_sample((const double *)psi, n, seed, traj, circ, n_samples, e0, e1, samples,
                       sample_margins) == 0 ? 0 : -2;
    if (psi_out) memcpy(psi_out, psi, sizeof(cplx) * dim);
    free(psi);
    return rc;
}
