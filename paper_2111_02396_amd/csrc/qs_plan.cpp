// Host-side planning: Kraus bounds, greedy gate fusion, fused matrices.
#include "qs_plan.h"

#include <algorithm>
#include <cmath>
#include <limits>

namespace qs {

namespace {

// Eigenvalues of a real symmetric m x m matrix by cyclic Jacobi rotations.
void jacobi_symmetric(int m, std::vector<double> &a, std::vector<double> &eig) {
    auto at = [&](int r, int c) -> double & { return a[size_t(r) * m + c]; };
    double scale = 0.0;
    for (double v : a) scale = std::max(scale, std::fabs(v));
    const double tiny = scale * 1e-300 + std::numeric_limits<double>::min();
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) off += at(p, q) * at(p, q);
        if (off <= (scale * scale) * 1e-34 || off == 0.0) break;
        for (int p = 0; p < m; ++p) {
            for (int q = p + 1; q < m; ++q) {
                const double apq = at(p, q);
                if (std::fabs(apq) <= tiny) continue;
                const double theta = (at(q, q) - at(p, p)) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0);
                const double s = t * c;
                for (int r = 0; r < m; ++r) {  // columns p, q
                    const double arp = at(r, p), arq = at(r, q);
                    at(r, p) = c * arp - s * arq;
                    at(r, q) = s * arp + c * arq;
                }
                for (int r = 0; r < m; ++r) {  // rows p, q
                    const double apr = at(p, r), aqr = at(q, r);
                    at(p, r) = c * apr - s * aqr;
                    at(q, r) = s * apr + c * aqr;
                }
            }
        }
    }
    eig.resize(m);
    for (int i = 0; i < m; ++i) eig[i] = at(i, i);
}

}  // namespace

double hermitian_min_eigenvalue(int d, const cd *A) {
    const int m = 2 * d;
    std::vector<double> a(size_t(m) * m);
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            const cd v = A[r * d + c];
            a[size_t(r) * m + c] = v.real();
            a[size_t(r) * m + c + d] = -v.imag();
            a[size_t(r + d) * m + c] = v.imag();
            a[size_t(r + d) * m + c + d] = v.real();
        }
    // symmetrise against rounding in the caller's Hermitian input
    for (int r = 0; r < m; ++r)
        for (int c = r + 1; c < m; ++c) {
            const double s = 0.5 * (a[size_t(r) * m + c] + a[size_t(c) * m + r]);
            a[size_t(r) * m + c] = a[size_t(c) * m + r] = s;
        }
    std::vector<double> eig;
    jacobi_symmetric(m, a, eig);
    return *std::min_element(eig.begin(), eig.end());
}

void gram(int d, const cd *K, cd *G) {
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            cd s = 0.0;
            for (int m = 0; m < d; ++m) s += std::conj(K[m * d + a]) * K[m * d + b];
            G[a * d + b] = s;
        }
}

bool is_identity_multiple(int d, const cd *M, double tol, cd *scalar_out) {
    const cd c = M[0];
    for (int r = 0; r < d; ++r)
        for (int col = 0; col < d; ++col) {
            const cd expect = r == col ? c : cd(0.0);
            if (std::abs(M[r * d + col] - expect) > tol) return false;
        }
    if (scalar_out) *scalar_out = c;
    return true;
}

void kraus_bounds(int k, int n_kraus, const cd *kraus, double *pbar, bool *mixture) {
    const int d = 1 << k;
    std::vector<cd> G(size_t(d) * d);
    bool mix = true;
    for (int i = 0; i < n_kraus; ++i) {
        gram(d, kraus + size_t(i) * d * d, G.data());
        const double lam = hermitian_min_eigenvalue(d, G.data());
        pbar[i] = lam > 0.0 ? lam : 0.0;
        double tr = 0.0;
        for (int j = 0; j < d; ++j) tr += G[j * d + j].real();
        const double c = tr / d;
        for (int r = 0; r < d && mix; ++r)
            for (int col = 0; col < d; ++col) {
                const cd expect = r == col ? cd(c) : cd(0.0);
                if (std::abs(G[r * d + col] - expect) > 1e-12) {
                    mix = false;
                    break;
                }
            }
    }
    *mixture = mix;
}

std::vector<Block> fuse_greedy(int n_qubits, const std::vector<PlanOp> &ops, int max_fuse,
                               std::vector<int> *op_block) {
    const int n_ops = int(ops.size());
    std::vector<std::vector<int>> on_qubit(n_qubits);
    for (int o = 0; o < n_ops; ++o)
        for (int j = 0; j < ops[o].k; ++j) on_qubit[ops[o].q[j]].push_back(o);
    std::vector<size_t> head(n_qubits, 0);
    std::vector<char> taken(n_ops, 0);
    if (op_block) op_block->assign(n_ops, -1);

    auto first_open = [&](int q) -> int {
        auto &lst = on_qubit[q];
        size_t &h = head[q];
        while (h < lst.size() && taken[lst[h]]) ++h;
        return h < lst.size() ? lst[h] : -1;
    };
    auto ready = [&](int o) -> bool {
        for (int j = 0; j < ops[o].k; ++j)
            if (first_open(ops[o].q[j]) != o) return false;
        return true;
    };

    std::vector<Block> blocks;
    for (int seed = 0; seed < n_ops; ++seed) {
        if (taken[seed]) continue;
        Block b;
        bool in_set[64] = {false};
        int qs[64];
        int nq = 0;
        auto add = [&](int o) {
            taken[o] = 1;
            b.ops.push_back(o);
            for (int j = 0; j < ops[o].k; ++j) {
                const int q = ops[o].q[j];
                if (!in_set[q]) {
                    in_set[q] = true;
                    qs[nq++] = q;
                }
            }
        };
        add(seed);
        const int limit = std::max(max_fuse, ops[seed].k);
        for (;;) {
            int best = -1;
            int best_growth = 0;
            for (int i = 0; i < nq; ++i) {
                const int c = first_open(qs[i]);
                if (c < 0 || !ready(c)) continue;
                int growth = 0;
                for (int j = 0; j < ops[c].k; ++j) growth += in_set[ops[c].q[j]] ? 0 : 1;
                if (nq + growth > limit) continue;
                const bool better = best < 0 || (growth == 0 && best_growth > 0) ||
                                    ((growth == 0) == (best_growth == 0) && c < best);
                if (better) {
                    best = c;
                    best_growth = growth;
                }
            }
            if (best < 0) break;
            add(best);
        }
        std::sort(b.ops.begin(), b.ops.end());
        std::sort(qs, qs + nq);
        b.k = nq;
        for (int i = 0; i < nq; ++i) b.q[i] = qs[i];
        blocks.push_back(std::move(b));
    }
    merge_subset_blocks(blocks);
    merge_cheaper_blocks(blocks, std::max(max_fuse, 1));
    if (op_block)
        for (size_t bi = 0; bi < blocks.size(); ++bi)
            for (int o : blocks[bi].ops) (*op_block)[o] = int(bi);
    return blocks;
}

void merge_subset_blocks(std::vector<Block> &blocks) {
    auto touches = [](const Block &a, const Block &b) {
        for (int i = 0; i < a.k; ++i)
            for (int j = 0; j < b.k; ++j)
                if (a.q[i] == b.q[j]) return true;
        return false;
    };
    auto subset = [](const Block &a, const Block &b) {  // qubits(a) within qubits(b)
        for (int i = 0; i < a.k; ++i) {
            bool found = false;
            for (int j = 0; j < b.k; ++j) found |= a.q[i] == b.q[j];
            if (!found) return false;
        }
        return true;
    };
    auto fold = [&](size_t from, size_t into) {
        Block &dst = blocks[into];
        dst.ops.insert(dst.ops.end(), blocks[from].ops.begin(), blocks[from].ops.end());
        std::sort(dst.ops.begin(), dst.ops.end());
        blocks.erase(blocks.begin() + std::ptrdiff_t(from));
    };
    size_t i = 0;
    while (i < blocks.size()) {
        bool merged = false;
        // the next block that shares a qubit with block i
        for (size_t j = i + 1; j < blocks.size(); ++j) {
            if (!touches(blocks[j], blocks[i])) continue;
            if (subset(blocks[i], blocks[j])) {
                fold(i, j);
                merged = true;
            }
            break;
        }
        if (!merged) {
            // the previous block that shares a qubit with block i
            for (size_t j = i; j-- > 0;) {
                if (!touches(blocks[j], blocks[i])) continue;
                if (subset(blocks[i], blocks[j])) {
                    fold(i, j);
                    merged = true;
                }
                break;
            }
        }
        if (!merged) ++i;  // after a fold, index i holds the next block
    }
}

int union_qubits(const std::vector<int> &members, const std::vector<PlanOp> &ops, int *q_out) {
    int nq = 0;
    for (int o : members)
        for (int j = 0; j < ops[o].k; ++j) {
            const int q = ops[o].q[j];
            bool seen = false;
            for (int i = 0; i < nq; ++i) seen |= q_out[i] == q;
            if (!seen) q_out[nq++] = q;
        }
    std::sort(q_out, q_out + nq);
    return nq;
}

void fused_matrix(int k, const int *q, const std::vector<int> &members,
                  const std::vector<PlanOp> &ops, const std::vector<const cd *> &mats, cd *out) {
    const int D = 1 << k;
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) out[r * D + c] = r == c ? cd(1.0) : cd(0.0);
    cd v[32], w[32];
    for (int o : members) {
        const cd *U = mats[o];
        if (!U) continue;
        const PlanOp &op = ops[o];
        const int ko = op.k, d = 1 << ko;
        int lp[5], lps[5];
        for (int j = 0; j < ko; ++j) {
            lp[j] = int(std::find(q, q + k, op.q[j]) - q);
            lps[j] = lp[j];
        }
        std::sort(lps, lps + ko);
        int off[32];
        for (int j = 0; j < d; ++j) {
            int x = 0;
            for (int b = 0; b < ko; ++b)
                if ((j >> b) & 1) x |= 1 << lp[b];
            off[j] = x;
        }
        const int groups = D >> ko;
        for (int g = 0; g < groups; ++g) {
            int base = g;
            for (int b = 0; b < ko; ++b) {
                const int p = lps[b];
                base = ((base >> p) << (p + 1)) | (base & ((1 << p) - 1));
            }
            for (int c = 0; c < D; ++c) {
                for (int j = 0; j < d; ++j) v[j] = out[(base + off[j]) * D + c];
                for (int j = 0; j < d; ++j) {
                    cd s = 0.0;
                    for (int l = 0; l < d; ++l) s += U[j * d + l] * v[l];
                    w[j] = s;
                }
                for (int j = 0; j < d; ++j) out[(base + off[j]) * D + c] = w[j];
            }
        }
    }
}

void to_ascending_order(int k, const int *t, const cd *in, cd *out, int *t_sorted) {
    const int D = 1 << k;
    int order[5];
    for (int j = 0; j < k; ++j) order[j] = j;
    std::sort(order, order + k, [&](int a, int b) { return t[a] < t[b]; });
    for (int s = 0; s < k; ++s) t_sorted[s] = t[order[s]];
    // original bit order[s] -> sorted bit s
    auto map = [&](int x) {
        int y = 0;
        for (int s = 0; s < k; ++s)
            if ((x >> order[s]) & 1) y |= 1 << s;
        return y;
    };
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) out[map(r) * D + map(c)] = in[r * D + c];
}

std::vector<Sweep> group_sweeps(int n_qubits, const std::vector<Block> &blocks, int max_bits,
                                int low_bits, int max_blocks, int mat_budget,
                                const int *slot_per_k, bool search) {
    const int nb = int(blocks.size());
    // predecessor counts and successor lists from per-qubit chains
    std::vector<int> last(n_qubits, -1);
    std::vector<int> npred(nb, 0);
    std::vector<std::vector<int>> succ(nb);
    for (int b = 0; b < nb; ++b) {
        for (int i = 0; i < blocks[b].k; ++i) {
            const int q = blocks[b].q[i];
            const int p = last[q];
            if (p >= 0 && (succ[p].empty() || succ[p].back() != b)) {
                succ[p].push_back(b);
                ++npred[b];
            }
            last[q] = b;
        }
    }
    std::vector<int> ready;
    for (int b = 0; b < nb; ++b)
        if (npred[b] == 0) ready.push_back(b);
    const int low = std::min(low_bits, n_qubits);

    // Fill one sweep greedily: repeatedly take the ready block that adds the
    // fewest new bits (ties: earliest), starting with `first` (if >= 0).
    // Works on copies of the ready list and predecessor counts; returns the
    // blocks taken in order and their total cost.
    struct Fill {
        std::vector<int> taken;
        std::vector<char> in;
        double cost = 0.0;
    };
    auto fill = [&](int first, std::vector<int> rdy, std::vector<int> &np) {
        Fill f;
        f.in.assign(n_qubits, 0);
        int nbits = 0;
        for (int q = 0; q < low; ++q) {
            f.in[q] = 1;
            ++nbits;
        }
        int mats = 0;
        auto take = [&](int pos) {
            const int b = rdy[pos];
            rdy.erase(rdy.begin() + pos);
            f.taken.push_back(b);
            f.cost += block_cost(blocks[b].k);
            mats += slot_per_k[blocks[b].k];
            for (int j = 0; j < blocks[b].k; ++j) {
                const int q = blocks[b].q[j];
                if (!f.in[q]) {
                    f.in[q] = 1;
                    ++nbits;
                }
            }
            for (int s2 : succ[b])
                if (--np[s2] == 0) rdy.push_back(s2);
        };
        auto fits = [&](int b, int *growth) {
            int g = 0;
            for (int j = 0; j < blocks[b].k; ++j) g += f.in[blocks[b].q[j]] ? 0 : 1;
            *growth = g;
            return nbits + g <= max_bits && mats + slot_per_k[blocks[b].k] <= mat_budget;
        };
        if (first >= 0) {
            int g;
            for (int i = 0; i < int(rdy.size()); ++i)
                if (rdy[i] == first) {
                    if (fits(first, &g)) take(i);
                    break;
                }
        }
        for (;;) {
            if (int(f.taken.size()) >= max_blocks) break;
            int best = -1, best_pos = -1, best_growth = 1 << 30;
            for (int i = 0; i < int(rdy.size()); ++i) {
                int g;
                if (!fits(rdy[i], &g)) continue;
                if (g < best_growth || (g == best_growth && rdy[i] < best)) {
                    best = rdy[i];
                    best_pos = i;
                    best_growth = g;
                }
            }
            if (best < 0) break;
            take(best_pos);
        }
        return f;
    };

    std::vector<Sweep> out;
    int done = 0;
    while (done < nb) {
        // every ready block as the first pick (plus the plain greedy); keep
        // the fill that absorbs the most block cost
        Fill best;
        best.cost = -1.0;
        std::vector<int> cand;
        if (search) cand = ready;
        cand.push_back(-1);
        for (int c : cand) {
            std::vector<int> np = npred;
            Fill f = fill(c, ready, np);
            if (f.cost > best.cost + 1e-9) best = std::move(f);
        }
        Sweep sw;
        if (best.taken.empty()) {
            // no ready block fits even an empty tile: it gets a sweep of its own,
            // wider than max_bits (the caller applies such sweeps block by block)
            int b = ready[0];
            for (int r : ready) b = std::min(b, r);
            best.taken.push_back(b);
            best.in.assign(n_qubits, 0);
            for (int q = 0; q < low; ++q) best.in[q] = 1;
            for (int j = 0; j < blocks[b].k; ++j) best.in[blocks[b].q[j]] = 1;
        }
        // commit: the taken blocks leave the ready list, their successors join
        for (int b : best.taken) {
            ready.erase(std::find(ready.begin(), ready.end(), b));
            sw.blocks.push_back(b);
            ++done;
            for (int s2 : succ[b])
                if (--npred[s2] == 0) ready.push_back(s2);
        }
        for (int q = 0; q < n_qubits; ++q)
            if (best.in[q]) sw.bits.push_back(q);
        out.push_back(std::move(sw));
    }
    return out;
}

std::vector<Sweep> group_sweeps_best(int n_qubits, const std::vector<Block> &blocks, int max_bits,
                                     int low_bits, int max_blocks, int mat_budget,
                                     const int *slot_per_k, int restarts, uint64_t seed) {
    std::vector<Sweep> best = group_sweeps(n_qubits, blocks, max_bits, low_bits, max_blocks,
                                           mat_budget, slot_per_k, true);
    if (restarts <= 0 || best.size() <= 1) return best;
    for (const auto &sw : best)
        if (int(sw.bits.size()) > max_bits) return best;  // a block that fits no tile: keep as is
    const int nb = int(blocks.size());
    std::vector<int> last(n_qubits, -1), npred0(nb, 0);
    std::vector<std::vector<int>> succ(nb);
    for (int b = 0; b < nb; ++b)
        for (int i = 0; i < blocks[b].k; ++i) {
            const int q = blocks[b].q[i], p = last[q];
            if (p >= 0 && (succ[p].empty() || succ[p].back() != b)) {
                succ[p].push_back(b);
                ++npred0[b];
            }
            last[q] = b;
        }
    const int low = std::min(low_bits, n_qubits);
    uint64_t state = seed;
    auto draw = [&state](size_t m) {  // splitmix64, reduced to [0, m)
        uint64_t z = (state += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return size_t((z ^ (z >> 31)) % m);
    };
    std::vector<int> npred, ready, cands;
    std::vector<char> in(n_qubits, 0);
    for (int r = 0; r < restarts; ++r) {
        npred = npred0;
        ready.clear();
        for (int b = 0; b < nb; ++b)
            if (npred[b] == 0) ready.push_back(b);
        std::vector<Sweep> cur;
        int done = 0;
        bool ok = true;
        while (done < nb) {
            if (cur.size() + 1 >= best.size()) {  // cannot end with fewer sweeps
                ok = false;
                break;
            }
            std::fill(in.begin(), in.end(), 0);
            int nbits = 0, mats = 0;
            for (int q = 0; q < low; ++q) {
                in[q] = 1;
                ++nbits;
            }
            Sweep sw;
            for (;;) {
                if (int(sw.blocks.size()) >= max_blocks) break;
                // the sweep's first block: any ready block that fits; later
                // ones: the least qubit growth, ties drawn at random
                cands.clear();
                int least = 1 << 30;
                for (int i = 0; i < int(ready.size()); ++i) {
                    const Block &B = blocks[ready[i]];
                    int g = 0;
                    for (int j = 0; j < B.k; ++j) g += in[B.q[j]] ? 0 : 1;
                    if (nbits + g > max_bits || mats + slot_per_k[B.k] > mat_budget) continue;
                    const int key = sw.blocks.empty() ? 0 : g;
                    if (key < least) {
                        least = key;
                        cands.clear();
                    }
                    if (key == least) cands.push_back(i);
                }
                if (cands.empty()) break;
                const int pos = cands[draw(cands.size())];
                const int b = ready[pos];
                ready.erase(ready.begin() + pos);
                sw.blocks.push_back(b);
                ++done;
                mats += slot_per_k[blocks[b].k];
                for (int j = 0; j < blocks[b].k; ++j)
                    if (!in[blocks[b].q[j]]) {
                        in[blocks[b].q[j]] = 1;
                        ++nbits;
                    }
                for (int s2 : succ[b])
                    if (--npred[s2] == 0) ready.push_back(s2);
            }
            if (sw.blocks.empty()) {
                ok = false;
                break;
            }
            for (int q = 0; q < n_qubits; ++q)
                if (in[q]) sw.bits.push_back(q);
            cur.push_back(std::move(sw));
        }
        if (ok && cur.size() < best.size()) best = std::move(cur);
    }
    return best;
}

double block_cost(int k) {
    // relative cost of one block applied to a tile in LDS by width: µs per
    // 2^24 amplitudes, measured on gfx950 with 13-bit tiles (barrier and read
    // latency make one-qubit blocks cost about 40 % of a four-qubit one)
    static const double c[6] = {0.0, 5.8, 9.1, 10.7, 14.5, 45.0};
    return k >= 1 && k <= 5 ? c[k] : 1e9;
}

void merge_cheaper_blocks(std::vector<Block> &blocks, int max_fuse) {
    constexpr size_t kWindow = 8;  // blocks looked ahead of each block
    auto shares = [](const Block &a, const Block &b) {
        for (int i = 0; i < a.k; ++i)
            for (int j = 0; j < b.k; ++j)
                if (a.q[i] == b.q[j]) return true;
        return false;
    };
    auto unite = [](const Block &a, const Block &b, int *q) {
        int nq = 0;
        for (int i = 0; i < a.k; ++i) q[nq++] = a.q[i];
        for (int j = 0; j < b.k; ++j) {
            bool seen = false;
            for (int i = 0; i < a.k; ++i) seen |= b.q[j] == a.q[i];
            if (!seen) q[nq++] = b.q[j];
        }
        std::sort(q, q + nq);
        return nq;
    };
    bool changed = true;
    while (changed) {
        changed = false;
        for (size_t i = 0; i < blocks.size() && !changed; ++i) {
            for (size_t j = i + 1; j < blocks.size() && j <= i + kWindow && !changed; ++j) {
                if (!shares(blocks[i], blocks[j])) continue;
                int q[10];
                const int nq = unite(blocks[i], blocks[j], q);
                if (nq > max_fuse || nq > 5) continue;
                if (!(block_cost(nq) < block_cost(blocks[i].k) + block_cost(blocks[j].k))) continue;
                // blocks strictly between i and j must not touch i's qubits (the
                // merged block takes j's place) or j's (it takes i's place)
                bool clear_i = true, clear_j = true;
                for (size_t z = i + 1; z < j; ++z) {
                    clear_i = clear_i && !shares(blocks[z], blocks[i]);
                    clear_j = clear_j && !shares(blocks[z], blocks[j]);
                }
                if (!clear_i && !clear_j) continue;
                const size_t keep = clear_i ? j : i, drop = clear_i ? i : j;
                Block &dst = blocks[keep];
                dst.ops.insert(dst.ops.end(), blocks[drop].ops.begin(), blocks[drop].ops.end());
                std::sort(dst.ops.begin(), dst.ops.end());
                dst.k = nq;
                for (int t = 0; t < 5; ++t) dst.q[t] = t < nq ? q[t] : 0;
                blocks.erase(blocks.begin() + std::ptrdiff_t(drop));
                changed = true;
            }
        }
    }
}

}  // namespace qs
