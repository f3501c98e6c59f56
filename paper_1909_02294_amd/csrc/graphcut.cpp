// Depth optimisation on the host: Eq. (1) minimised by alpha-expansion graph
// cuts over segment nodes (Sec. III-B), with the label-partitioned threads
// and pairwise merging of Sec. IV-A.
//
// Every energy term is rounded to an integer multiple of 1/quantum, so the
// maximum flows are exact.  Each move takes the canonical minimum cut: its
// source side (segments that keep their label) is the set of nodes reachable
// from the source in the residual graph, found by a search after the flow.
// That set is the same for every maximum flow, so the result does not depend
// on the max-flow algorithm or on the order of augmentations.
//
// Max-flow: the search-tree augmenting-path method of Boykov and Kolmogorov
// (IEEE TPAMI 26(9), 2004): two trees grown from the terminals, augmentation
// along the path where they meet, and adoption of orphaned nodes.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <thread>
#include <vector>

#include "../../include/ivde.h"
#include "host_common.h"

using namespace ivde;

namespace {

// ------------------------------------------------------------------ max-flow
class MaxFlow {
public:
    void reset(int n)
    {
        n_ = n;
        tr_.assign(n, 0);
        edges_.clear();
        flow_ = 0;
    }
    // cap_source: cost of putting i on the sink side; cap_sink: on the source side
    void add_tweights(int i, int64_t cap_source, int64_t cap_sink)
    {
        const int64_t d = std::min(cap_source, cap_sink);
        flow_ += d;
        tr_[i] += (cap_source - d) - (cap_sink - d);
    }
    // arc i->j of capacity c (cut when i is on the source side, j on the sink side)
    void add_edge(int i, int j, int64_t c) { edges_.push_back({i, j, c}); }
    int64_t solve();
    // nodes reachable from the source in the residual graph (after solve)
    void source_side(std::vector<uint8_t> &out) const;

private:
    struct Edge {
        int i, j;
        int64_t c;
    };
    static constexpr int kTerminal = -2, kOrphan = -3, kNone = -1;
    void build_arcs();
    void set_active(int i)
    {
        if (!queued_[i]) {
            queued_[i] = 1;
            queue_.push_back(i);
        }
    }
    void augment(int mid);
    void adopt();

    int n_ = 0;
    std::vector<Edge> edges_;
    // arcs in CSR order: node i owns [first_[i], first_[i + 1])
    std::vector<int> first_, head_, sister_;
    std::vector<int64_t> rcap_, tr_;
    int64_t flow_ = 0;
    // search state
    std::vector<int> parent_, ts_, dist_;
    std::vector<uint8_t> sink_, queued_;
    std::vector<int> queue_;
    std::deque<int> orphans_;   // taken from the front; freed nodes' children join at the back
    size_t qhead_ = 0;
    int time_ = 0;
};

void MaxFlow::build_arcs()
{
    first_.assign(n_ + 1, 0);
    for (const Edge &e : edges_) {
        ++first_[e.i + 1];
        ++first_[e.j + 1];
    }
    for (int i = 0; i < n_; ++i) first_[i + 1] += first_[i];
    const size_t na = 2 * edges_.size();
    head_.resize(na);
    sister_.resize(na);
    rcap_.resize(na);
    std::vector<int> pos(first_.begin(), first_.end() - 1);
    for (const Edge &e : edges_) {
        const int a = pos[e.i]++, b = pos[e.j]++;
        head_[a] = e.j;
        rcap_[a] = e.c;
        sister_[a] = b;
        head_[b] = e.i;
        rcap_[b] = 0;
        sister_[b] = a;
    }
}

int64_t MaxFlow::solve()
{
    build_arcs();
    // push along every path source -> i -> j -> sink before the tree search
    for (int i = 0; i < n_; ++i) {
        if (tr_[i] <= 0) continue;
        for (int a = first_[i]; a < first_[i + 1] && tr_[i] > 0; ++a) {
            const int j = head_[a];
            if (tr_[j] >= 0 || rcap_[a] <= 0) continue;
            const int64_t f = std::min(std::min(tr_[i], rcap_[a]), -tr_[j]);
            tr_[i] -= f;
            tr_[j] += f;
            rcap_[a] -= f;
            rcap_[sister_[a]] += f;
            flow_ += f;
        }
    }
    parent_.assign(n_, kNone);
    ts_.assign(n_, 0);
    dist_.assign(n_, 0);
    sink_.assign(n_, 0);
    queued_.assign(n_, 0);
    queue_.clear();
    qhead_ = 0;
    orphans_.clear();
    time_ = 0;
    for (int i = 0; i < n_; ++i) {
        if (tr_[i] != 0) {
            parent_[i] = kTerminal;
            sink_[i] = tr_[i] < 0;
            dist_[i] = 1;
            set_active(i);
        }
    }
    int cur = -1;
    for (;;) {
        int i = cur;
        cur = -1;
        if (i < 0) {
            // next active node that is still in a tree
            while (qhead_ < queue_.size()) {
                const int k = queue_[qhead_++];
                queued_[k] = 0;
                if (parent_[k] != kNone) {
                    i = k;
                    break;
                }
            }
            if (qhead_ > 4096 && qhead_ * 2 > queue_.size()) {
                queue_.erase(queue_.begin(), queue_.begin() + (ptrdiff_t)qhead_);
                qhead_ = 0;
            }
            if (i < 0) break;
        }
        // growth
        int mid = -1;
        const int a0 = first_[i], a1 = first_[i + 1];
        if (!sink_[i]) {
            for (int a = a0; a < a1; ++a) {
                if (rcap_[a] <= 0) continue;
                const int j = head_[a];
                if (parent_[j] == kNone) {
                    sink_[j] = 0;
                    parent_[j] = sister_[a];
                    ts_[j] = ts_[i];
                    dist_[j] = dist_[i] + 1;
                    set_active(j);
                } else if (sink_[j]) {
                    mid = a;
                    break;
                } else if (ts_[j] <= ts_[i] && dist_[j] > dist_[i]) {
                    parent_[j] = sister_[a];
                    ts_[j] = ts_[i];
                    dist_[j] = dist_[i] + 1;
                }
            }
        } else {
            for (int a = a0; a < a1; ++a) {
                if (rcap_[sister_[a]] <= 0) continue;
                const int j = head_[a];
                if (parent_[j] == kNone) {
                    sink_[j] = 1;
                    parent_[j] = sister_[a];
                    ts_[j] = ts_[i];
                    dist_[j] = dist_[i] + 1;
                    set_active(j);
                } else if (!sink_[j]) {
                    mid = sister_[a];
                    break;
                } else if (ts_[j] <= ts_[i] && dist_[j] > dist_[i]) {
                    parent_[j] = sister_[a];
                    ts_[j] = ts_[i];
                    dist_[j] = dist_[i] + 1;
                }
            }
        }
        ++time_;
        if (mid >= 0) {
            augment(mid);
            adopt();
            if (parent_[i] != kNone) cur = i;   // i may grow further
        }
    }
    return flow_;
}

// Push the bottleneck along source -> ... -> tail(mid) -> head(mid) -> ... -> sink.
// A node's parent arc leads from the node towards its tree's root.
void MaxFlow::augment(int mid)
{
    int64_t b = rcap_[mid];
    int i;
    for (i = head_[sister_[mid]];; i = head_[parent_[i]]) {
        const int a = parent_[i];
        if (a == kTerminal) break;
        b = std::min(b, rcap_[sister_[a]]);
    }
    b = std::min(b, tr_[i]);
    for (i = head_[mid];; i = head_[parent_[i]]) {
        const int a = parent_[i];
        if (a == kTerminal) break;
        b = std::min(b, rcap_[a]);
    }
    b = std::min(b, -tr_[i]);

    rcap_[sister_[mid]] += b;
    rcap_[mid] -= b;
    for (i = head_[sister_[mid]];;) {
        const int a = parent_[i];
        if (a == kTerminal) {
            tr_[i] -= b;
            if (tr_[i] == 0) {
                parent_[i] = kOrphan;
                orphans_.push_front(i);
            }
            break;
        }
        rcap_[a] += b;
        rcap_[sister_[a]] -= b;
        const int up = head_[a];
        if (rcap_[sister_[a]] == 0) {
            parent_[i] = kOrphan;
            orphans_.push_front(i);
        }
        i = up;
    }
    for (i = head_[mid];;) {
        const int a = parent_[i];
        if (a == kTerminal) {
            tr_[i] += b;
            if (tr_[i] == 0) {
                parent_[i] = kOrphan;
                orphans_.push_front(i);
            }
            break;
        }
        rcap_[sister_[a]] += b;
        rcap_[a] -= b;
        const int down = head_[a];
        if (rcap_[a] == 0) {
            parent_[i] = kOrphan;
            orphans_.push_front(i);
        }
        i = down;
    }
    flow_ += b;
}

// Give each orphan a new parent in its tree whose path reaches the terminal,
// or free it (its children become orphans, its neighbours active).
void MaxFlow::adopt()
{
    while (!orphans_.empty()) {
        const int i = orphans_.front();
        orphans_.pop_front();
        const bool sink = sink_[i];
        int best = -1;
        int dmin = INT_MAX;
        const int a0 = first_[i], a1 = first_[i + 1];
        for (int a = a0; a < a1; ++a) {
            // residual towards i (source tree) or away from i (sink tree)
            if ((sink ? rcap_[a] : rcap_[sister_[a]]) <= 0) continue;
            const int j = head_[a];
            if (sink_[j] != sink || parent_[j] == kNone) continue;
            // does j's path reach the terminal?
            int d = 0;
            int k = j;
            for (;;) {
                if (ts_[k] == time_) {
                    d += dist_[k];
                    break;
                }
                const int pa = parent_[k];
                ++d;
                if (pa == kTerminal) {
                    ts_[k] = time_;
                    dist_[k] = 1;
                    break;
                }
                if (pa == kOrphan) {
                    d = INT_MAX;
                    break;
                }
                k = head_[pa];
            }
            if (d == INT_MAX) continue;
            if (d < dmin) {
                best = a;
                dmin = d;
            }
            for (k = j; ts_[k] != time_; k = head_[parent_[k]]) {
                ts_[k] = time_;
                dist_[k] = d--;
            }
        }
        if (best >= 0) {
            parent_[i] = best;
            ts_[i] = time_;
            dist_[i] = dmin + 1;
            continue;
        }
        // free i
        for (int a = a0; a < a1; ++a) {
            const int j = head_[a];
            if (sink_[j] != sink || parent_[j] == kNone) continue;
            if ((sink ? rcap_[a] : rcap_[sister_[a]]) > 0) set_active(j);
            const int pa = parent_[j];
            if (pa != kTerminal && pa != kOrphan && head_[pa] == i) {
                parent_[j] = kOrphan;
                orphans_.push_back(j);
            }
        }
        parent_[i] = kNone;
    }
}

// When the search stops, no source-tree node has a residual arc to a node
// outside the tree (that node would still be active) and every tree node
// reaches the source along its parent arcs, so the source tree is exactly
// the set of nodes reachable from the source in the residual graph.
void MaxFlow::source_side(std::vector<uint8_t> &out) const
{
    out.resize(n_);
    for (int i = 0; i < n_; ++i) out[i] = parent_[i] != kNone && !sink_[i];
}

// ------------------------------------------------------------------ energy
int64_t quantize(double x, double q) { return (int64_t)std::llround(x * q); }

// The term tables are stored level-major ([L][rows] and [L][rows][2]), so
// that a move towards one level reads them in row order.
struct Model {
    int64_t rows = 0;
    int L = 0;
    std::vector<int64_t> UT;         // [L][rows] quantised unary, or empty
    std::vector<int32_t> HT;         // [L][rows][2] window hits (-1: none), or empty
    std::vector<int64_t> RT;         // [L][rows][2] quantised rewards (0 without a hit), or empty
    // adjacency as unordered pairs, listed from both ends: row r's pairs are
    // [poff[r], poff[r + 1]), weight = the sum of both ordered entries' weights
    std::vector<int64_t> poff;
    std::vector<int32_t> ptgt;
    std::vector<int64_t> pw;
    std::vector<int32_t> fixed;      // label or -1

    int64_t unary(int64_t r, int l) const { return UT.empty() ? 0 : UT[(size_t)l * rows + r]; }
    int32_t hit_at(int64_t r, int s, int l) const { return HT.empty() ? -1 : HT[((size_t)l * rows + r) * 2 + s]; }
    int64_t reward(int64_t r, int s, int l) const { return RT.empty() ? 0 : RT[((size_t)l * rows + r) * 2 + s]; }
    bool is_free(int64_t r) const { return fixed.empty() || fixed[r] < 0; }

    int64_t energy(const std::vector<int32_t> &d) const
    {
        int64_t e = 0;
        for (int64_t r = 0; r < rows; ++r) {
            const int l = d[r];
            e += unary(r, l);
            for (int s = 0; s < 2; ++s) {
                const int32_t h = hit_at(r, s, l);
                if (h >= 0 && d[h] == l) e += reward(r, s, l);
            }
            for (int64_t k = poff.empty() ? 0 : poff[r]; k < (poff.empty() ? 0 : poff[r + 1]); ++k)
                if (ptgt[k] > r) e += pw[k] * std::abs(l - d[ptgt[k]]);
        }
        return e;
    }
};

// Rows that may take level l in a merge: those whose candidate labels
// include l, bucketed by level.
struct Buckets {
    std::vector<int64_t> off;
    std::vector<int32_t> row;
};

// Alpha-expansion moves over one labelling.  Keeps an index from each row
// to the (row, slot) window terms whose current hit lands on it, so a move
// visits only the segments that may switch and the terms touching them.
class Mover {
public:
    explicit Mover(const Model &m) : M(m), node_(m.rows, -1), rev_(m.rows) {}

    void begin(const std::vector<int32_t> &d)
    {
        cu_.resize(M.rows);
        ch_.resize(2 * M.rows);
        cr_.resize(2 * M.rows);
        for (int64_t q = 0; q < M.rows; ++q) set_current(q, d[q]);
        for (auto &v : rev_) v.clear();
        for (int64_t q = 0; q < M.rows; ++q)
            for (int s = 0; s < 2; ++s) rev_add(q, s);
    }

    // Returns true (and updates d, e) when the canonical optimal move lowers the energy.
    bool move(std::vector<int32_t> &d, int64_t &e, int alpha, const std::vector<int32_t> *cand_a,
              const std::vector<int32_t> *cand_b, const Buckets *bk)
    {
        nodes_.clear();
        auto consider = [&](int64_t r) {
            if (!M.is_free(r) || d[r] == alpha || node_[r] >= 0) return;
            if (cand_a && (*cand_a)[r] != alpha && (*cand_b)[r] != alpha) return;
            node_[r] = (int)nodes_.size();
            nodes_.push_back(r);
        };
        if (bk) {
            for (int64_t k = bk->off[alpha]; k < bk->off[alpha + 1]; ++k) consider(bk->row[k]);
        } else {
            for (int64_t r = 0; r < M.rows; ++r) consider(r);
        }
        if (nodes_.empty()) return false;
        const int n = (int)nodes_.size();
        g_.reset(n);
        net_.assign(n, 0);
        pairs_.clear();
        auto lab = [&](int64_t r, int x) { return (x && node_[r] >= 0) ? alpha : d[r]; };
        auto unary1 = [&](int i, int64_t c0, int64_t c1) { net_[i] += c1 - c0; };
        bool nonsub = false;
        auto pair = [&](int i, int j, int64_t A, int64_t B, int64_t C, int64_t D) {
            // A + (C - A) x_i + (D - C) x_j + (B + C - A - D)(1 - x_i) x_j
            net_[i] += C - A;
            net_[j] += D - C;
            const int64_t w = B + C - A - D;
            if (w > 0) {
                g_.add_edge(i, j, w);
                pairs_.push_back({i, j, w});
            }
            if (w < 0) nonsub = true;
        };
        for (int ir = 0; ir < n; ++ir) {
            const int64_t r = nodes_[ir];
            const int dr = d[r];
            unary1(ir, cu_[r], M.unary(r, alpha));
            // r's own window terms: Rv [label_r = c][label_h = c] for its two candidates c
            for (int s = 0; s < 2; ++s) {
                for (int xr = 0; xr < 2; ++xr) {
                    const int c = xr ? alpha : dr;
                    const int32_t h = xr ? M.hit_at(r, s, alpha) : ch_[2 * r + s];
                    if (h < 0) continue;
                    const int64_t Rv = xr ? M.reward(r, s, alpha) : cr_[2 * r + s];
                    if (Rv == 0) continue;
                    const int ih = node_[h];
                    if (h == r) {
                        unary1(ir, xr == 0 ? Rv : 0, xr == 1 ? Rv : 0);
                    } else if (ih >= 0) {
                        int64_t t[2][2];
                        for (int a = 0; a < 2; ++a)
                            for (int b = 0; b < 2; ++b) t[a][b] = (a == xr && lab(h, b) == c) ? Rv : 0;
                        pair(ir, ih, t[0][0], t[0][1], t[1][0], t[1][1]);
                    } else {
                        const int64_t v = d[h] == c ? Rv : 0;
                        unary1(ir, xr == 0 ? v : 0, xr == 1 ? v : 0);
                    }
                }
            }
            // window terms of segments that keep their label and hit r
            for (uint64_t code : rev_[r]) {
                const int64_t q = (int64_t)(code >> 1);
                if (node_[q] >= 0) continue;   // a switchable q's terms are its own
                const int s = (int)(code & 1);
                const int c = d[q];
                const int64_t Rq = cr_[2 * q + s];
                unary1(ir, dr == c ? Rq : 0, alpha == c ? Rq : 0);
            }
            // intra-view pairs
            for (int64_t k = M.poff.empty() ? 0 : M.poff[r]; k < (M.poff.empty() ? 0 : M.poff[r + 1]); ++k) {
                const int64_t t = M.ptgt[k];
                const int64_t w = M.pw[k];
                const int it = node_[t];
                const int dt = d[t];
                if (it >= 0) {
                    if (t < r) continue;   // handled from t
                    pair(ir, it, w * std::abs(dr - dt), w * std::abs(dr - alpha), w * std::abs(alpha - dt), 0);
                } else {
                    unary1(ir, w * std::abs(dr - dt), w * std::abs(alpha - dt));
                }
            }
        }
        nonsub_ |= nonsub;
        for (int i = 0; i < n; ++i) {
            if (net_[i] > 0)
                g_.add_tweights(i, net_[i], 0);
            else if (net_[i] < 0)
                g_.add_tweights(i, 0, -net_[i]);
        }
        g_.solve();
        g_.source_side(side_);
        // energy change of the move, from its binary form
        int64_t delta = 0;
        bool any = false;
        for (int i = 0; i < n; ++i)
            if (!side_[i]) {
                delta += net_[i];
                any = true;
            }
        for (const PairEdge &pe : pairs_)
            if (side_[pe.i] && !side_[pe.j]) delta += pe.w;
        bool taken = false;
        if (any && delta < 0) {
            for (int i = 0; i < n; ++i)
                if (!side_[i]) {
                    const int64_t q = nodes_[i];
                    for (int s = 0; s < 2; ++s) rev_remove(q, s);
                    d[q] = alpha;
                    set_current(q, alpha);
                    for (int s = 0; s < 2; ++s) rev_add(q, s);
                }
            e += delta;
            taken = true;
        }
        for (int64_t r : nodes_) node_[r] = -1;
        return taken;
    }

    bool nonsubmodular() const { return nonsub_; }

private:
    struct PairEdge {
        int i, j;
        int64_t w;
    };
    // terms of row q at its current level
    void set_current(int64_t q, int l)
    {
        cu_[q] = M.unary(q, l);
        for (int s = 0; s < 2; ++s) {
            ch_[2 * q + s] = M.hit_at(q, s, l);
            cr_[2 * q + s] = M.reward(q, s, l);
        }
    }
    void rev_add(int64_t q, int s)
    {
        const int32_t h = ch_[2 * q + s];
        if (h >= 0 && cr_[2 * q + s] != 0) rev_[h].push_back(((uint64_t)q << 1) | (uint64_t)s);
    }
    void rev_remove(int64_t q, int s)
    {
        const int32_t h = ch_[2 * q + s];
        if (h < 0 || cr_[2 * q + s] == 0) return;
        auto &v = rev_[h];
        const uint64_t code = ((uint64_t)q << 1) | (uint64_t)s;
        for (size_t k = 0; k < v.size(); ++k)
            if (v[k] == code) {
                v[k] = v.back();
                v.pop_back();
                return;
            }
    }

    const Model &M;
    std::vector<int> node_;
    std::vector<int64_t> cu_;        // unary at the current level
    std::vector<int32_t> ch_;        // [rows][2] hits at the current level
    std::vector<int64_t> cr_;        // [rows][2] rewards at the current level
    std::vector<std::vector<uint64_t>> rev_;
    std::vector<int64_t> nodes_;
    std::vector<int64_t> net_;
    std::vector<PairEdge> pairs_;
    std::vector<uint8_t> side_;
    MaxFlow g_;
    bool nonsub_ = false;
};

struct Result {
    std::vector<int32_t> d;
    int64_t e = 0;
    std::vector<int> labels;
    int cycles = 0;
};

// Cycles of moves over `labels` in increasing order until a cycle changes nothing.
void expansion(const Model &M, Result &res, const std::vector<int> &labels, int max_cycles,
               const std::vector<int32_t> *cand_a, const std::vector<int32_t> *cand_b, bool &nonsub)
{
    Mover mv(M);
    mv.begin(res.d);
    res.e = M.energy(res.d);
    res.cycles = 0;
    Buckets bk;
    if (cand_a) {
        bk.off.assign(M.L + 1, 0);
        for (int64_t r = 0; r < M.rows; ++r) {
            ++bk.off[(*cand_a)[r] + 1];
            if ((*cand_b)[r] != (*cand_a)[r]) ++bk.off[(*cand_b)[r] + 1];
        }
        for (int l = 0; l < M.L; ++l) bk.off[l + 1] += bk.off[l];
        bk.row.resize(bk.off[M.L]);
        std::vector<int64_t> pos(bk.off.begin(), bk.off.end() - 1);
        for (int64_t r = 0; r < M.rows; ++r) {
            bk.row[pos[(*cand_a)[r]]++] = (int32_t)r;
            if ((*cand_b)[r] != (*cand_a)[r]) bk.row[pos[(*cand_b)[r]]++] = (int32_t)r;
        }
    }
    for (int c = 0; c < max_cycles; ++c) {
        ++res.cycles;
        bool changed = false;
        for (int alpha : labels) changed |= mv.move(res.d, res.e, alpha, cand_a, cand_b, cand_a ? &bk : nullptr);
        if (!changed) break;
    }
    nonsub |= mv.nonsubmodular();
}

std::vector<std::vector<int>> partition_labels(int L, int n, int partition)
{
    n = std::max(1, std::min(n, L));
    std::vector<std::vector<int>> subs(n);
    for (int k = 0; k < n; ++k) {
        if (partition == IVDE_PARTITION_BLOCKS) {
            for (int l = (int)((int64_t)k * L / n); l < (int)((int64_t)(k + 1) * L / n); ++l) subs[k].push_back(l);
        } else {
            for (int l = k; l < L; l += n) subs[k].push_back(l);
        }
    }
    subs.erase(std::remove_if(subs.begin(), subs.end(), [](const std::vector<int> &s) { return s.empty(); }),
               subs.end());
    return subs;
}

// Each free segment starts at the label of the subset with the lowest unary
// cost (the lowest such label); fixed segments at their own label.
void initial(const Model &M, const std::vector<int> &labels, std::vector<int32_t> &d)
{
    d.assign(M.rows, labels[0]);
    if (!M.UT.empty()) {
        std::vector<int64_t> best(M.rows);
        for (int64_t r = 0; r < M.rows; ++r) best[r] = M.unary(r, labels[0]);
        for (int l : labels)
            for (int64_t r = 0; r < M.rows; ++r) {
                const int64_t u = M.unary(r, l);
                if (u < best[r]) {
                    best[r] = u;
                    d[r] = l;
                }
            }
    }
    for (int64_t r = 0; r < M.rows; ++r)
        if (!M.is_free(r)) d[r] = M.fixed[r];
}

Result merge(const Model &M, const Result &A, const Result &B, int max_cycles, bool &nonsub)
{
    Result out;
    out.d = A.e <= B.e ? A.d : B.d;
    out.labels = A.labels;
    out.labels.insert(out.labels.end(), B.labels.begin(), B.labels.end());
    std::sort(out.labels.begin(), out.labels.end());
    out.labels.erase(std::unique(out.labels.begin(), out.labels.end()), out.labels.end());
    expansion(M, out, out.labels, max_cycles, &A.d, &B.d, nonsub);
    return out;
}

int build_threads() { return (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency())); }

ivde_status build_model(const ivde_energy *E, Model &M)
{
    if (!E || E->rows < 1 || E->num_labels < 1 || !(std::isfinite(E->quantum) && E->quantum > 0)) {
        set_error("energy: rows >= 1, num_labels >= 1 and a positive quantum are required");
        return IVDE_EINVAL;
    }
    if (E->rows >= ((int64_t)1 << 31)) {
        set_error("energy: too many rows");
        return IVDE_EINVAL;
    }
    if ((E->window_m == nullptr) != (E->window_hit == nullptr) ||
        (E->adj_offsets && (!E->adj_index || !E->adj_beta))) {
        set_error("energy: window_m and window_hit go together, as do offsets, index and beta");
        return IVDE_EINVAL;
    }
    const int64_t rows = E->rows;
    const int L = E->num_labels;
    const double q = E->quantum;
    const double limit = std::ldexp(1.0, 40);
    M.rows = rows;
    M.L = L;
    // level-major transposition in blocks of rows, spread over host threads
    constexpr int64_t kBlock = 64;
    const int64_t n_blocks = (rows + kBlock - 1) / kBlock;
    const int workers = (int)std::max<int64_t>(1, std::min<int64_t>(n_blocks, build_threads()));
    struct Bad {
        int kind = 0;   // 1 unary, 2 hit, 3 window value
        size_t at = 0;
        double value = 0;
    };
    std::vector<Bad> bad(workers);
    auto run = [&](auto &&body) {
        std::vector<std::thread> pool;
        for (int w = 0; w < workers; ++w)
            pool.emplace_back([&, w] {
                for (int64_t b = w; b < n_blocks; b += workers) {
                    const int64_t r0 = b * kBlock, r1 = std::min(rows, r0 + kBlock);
                    if (!body(r0, r1, bad[w])) return;
                }
            });
        for (auto &t : pool) t.join();
        for (const Bad &x : bad)
            if (x.kind) return x;
        return Bad{};
    };
    if (E->unary) {
        if (!std::isfinite(E->unary_weight)) {
            set_error("energy: unary_weight must be finite");
            return IVDE_EINVAL;
        }
        M.UT.resize((size_t)rows * L);
        const Bad x = run([&](int64_t r0, int64_t r1, Bad &bd) {
            for (int l = 0; l < L; ++l)
                for (int64_t r = r0; r < r1; ++r) {
                    const double u = E->unary_weight * (double)E->unary[(size_t)r * L + l];
                    if (!(std::fabs(u * q) < limit)) {
                        bd = {1, (size_t)r * L + l, u};
                        return false;
                    }
                    M.UT[(size_t)l * rows + r] = quantize(u, q);
                }
            return true;
        });
        if (x.kind) {
            set_error("energy: unary value %g too large for quantum %g", x.value, q);
            return IVDE_EINVAL;
        }
    }
    if (E->window_m) {
        M.HT.resize((size_t)rows * 2 * L);
        M.RT.resize((size_t)rows * 2 * L);
        const Bad x = run([&](int64_t r0, int64_t r1, Bad &bd) {
            for (int l = 0; l < L; ++l)
                for (int64_t r = r0; r < r1; ++r)
                    for (int sl = 0; sl < 2; ++sl) {
                        const size_t src = ((size_t)r * 2 + sl) * L + l;
                        const size_t dst = ((size_t)l * rows + r) * 2 + sl;
                        const int32_t h = E->window_hit[src];
                        if (h < -1 || h >= rows) {
                            bd = {2, src, (double)h};
                            return false;
                        }
                        M.HT[dst] = h;
                        if (h < 0) {
                            M.RT[dst] = 0;
                            continue;
                        }
                        const double v = std::min(0.0, (double)E->window_m[src] - (double)E->K);
                        if (!(std::fabs(v * q) < limit)) {
                            bd = {3, src, (double)E->window_m[src]};
                            return false;
                        }
                        M.RT[dst] = quantize(v, q);
                    }
            return true;
        });
        if (x.kind == 2) {
            set_error("energy: window_hit entry %zu (%d) outside [-1, rows)", x.at, (int)x.value);
            return IVDE_EINVAL;
        }
        if (x.kind == 3) {
            set_error("energy: window value %g too large for quantum %g", x.value, q);
            return IVDE_EINVAL;
        }
    }
    if (E->adj_offsets) {
        const int64_t *off = E->adj_offsets;
        if (off[0] != 0) {
            set_error("energy: adjacency offsets must start at 0");
            return IVDE_EINVAL;
        }
        for (int64_t r = 0; r < rows; ++r)
            if (off[r + 1] < off[r]) {
                set_error("energy: adjacency offsets decrease at row %lld", (long long)r);
                return IVDE_EINVAL;
            }
        // unordered pairs with the summed weight of both ordered entries
        struct P3 {
            int32_t a, b;
            int64_t w;
        };
        std::vector<P3> prs;
        prs.reserve((size_t)off[rows]);
        for (int64_t r = 0; r < rows; ++r)
            for (int64_t k = off[r]; k < off[r + 1]; ++k) {
                const int32_t t = E->adj_index[k];
                if (t < 0 || t >= rows) {
                    set_error("energy: adjacency entry %lld names row %d", (long long)k, t);
                    return IVDE_EINVAL;
                }
                const double v = (double)E->adj_beta[k] * q;
                if (!(E->adj_beta[k] >= 0.f) || !(v < limit / L)) {
                    set_error("energy: beta %g must be >= 0 and small enough for quantum %g",
                              (double)E->adj_beta[k], q);
                    return IVDE_EINVAL;
                }
                const int64_t w = quantize(E->adj_beta[k], q);
                if (t == r || w == 0) continue;
                prs.push_back({(int32_t)std::min<int64_t>(r, t), (int32_t)std::max<int64_t>(r, t), w});
            }
        std::sort(prs.begin(), prs.end(), [](const P3 &x, const P3 &y) { return x.a != y.a ? x.a < y.a : x.b < y.b; });
        size_t u = 0;
        for (size_t k = 0; k < prs.size(); ++k) {
            if (u > 0 && prs[u - 1].a == prs[k].a && prs[u - 1].b == prs[k].b)
                prs[u - 1].w += prs[k].w;
            else
                prs[u++] = prs[k];
        }
        prs.resize(u);
        M.poff.assign(rows + 1, 0);
        for (const P3 &p : prs) {
            ++M.poff[p.a + 1];
            ++M.poff[p.b + 1];
        }
        for (int64_t r = 0; r < rows; ++r) M.poff[r + 1] += M.poff[r];
        M.ptgt.resize(M.poff[rows]);
        M.pw.resize(M.poff[rows]);
        std::vector<int64_t> pos(M.poff.begin(), M.poff.end() - 1);
        for (const P3 &p : prs) {
            M.ptgt[pos[p.a]] = p.b;
            M.pw[pos[p.a]++] = p.w;
            M.ptgt[pos[p.b]] = p.a;
            M.pw[pos[p.b]++] = p.w;
        }
    }
    if (E->fixed_labels) {
        M.fixed.assign(E->fixed_labels, E->fixed_labels + rows);
        for (int64_t r = 0; r < rows; ++r)
            if (M.fixed[r] < -1 || M.fixed[r] >= L) {
                set_error("energy: fixed label of row %lld outside [-1, num_labels)", (long long)r);
                return IVDE_EINVAL;
            }
    }
    return IVDE_OK;
}

}  // namespace

extern "C" {

ivde_status ivde_energy_value(const ivde_energy *energy, const int32_t *labels, int64_t *energy_out)
{
    Model M;
    ivde_status st = build_model(energy, M);
    if (st != IVDE_OK) return st;
    if (!labels || !energy_out) {
        set_error("energy_value: labels and energy_out are required");
        return IVDE_EINVAL;
    }
    std::vector<int32_t> d(labels, labels + M.rows);
    for (int64_t r = 0; r < M.rows; ++r)
        if (d[r] < 0 || d[r] >= M.L) {
            set_error("energy_value: label of row %lld outside [0, num_labels)", (long long)r);
            return IVDE_EINVAL;
        }
    *energy_out = M.energy(d);
    return IVDE_OK;
}

ivde_status ivde_expansion(const ivde_energy *energy, int32_t *labels, const int32_t *label_list, int32_t n_list,
                           int32_t max_cycles, int64_t *energy_out, int32_t *cycles_out)
{
    Model M;
    ivde_status st = build_model(energy, M);
    if (st != IVDE_OK) return st;
    if (!labels || !label_list || n_list < 1 || max_cycles < 1) {
        set_error("expansion: labels, a non-empty label list and max_cycles >= 1 are required");
        return IVDE_EINVAL;
    }
    std::vector<int> ls(label_list, label_list + n_list);
    for (int l : ls)
        if (l < 0 || l >= M.L) {
            set_error("expansion: label %d outside [0, num_labels)", l);
            return IVDE_EINVAL;
        }
    std::sort(ls.begin(), ls.end());
    ls.erase(std::unique(ls.begin(), ls.end()), ls.end());
    Result res;
    res.d.assign(labels, labels + M.rows);
    for (int64_t r = 0; r < M.rows; ++r)
        if (res.d[r] < 0 || res.d[r] >= M.L || (!M.fixed.empty() && M.fixed[r] >= 0 && res.d[r] != M.fixed[r])) {
            set_error("expansion: label of row %lld outside [0, num_labels) or not its fixed label", (long long)r);
            return IVDE_EINVAL;
        }
    bool nonsub = false;
    expansion(M, res, ls, max_cycles, nullptr, nullptr, nonsub);
    if (nonsub) {
        set_error("expansion: a move was not submodular (negative adjacency weight or positive reward)");
        return IVDE_EINVAL;
    }
    if (M.energy(res.d) != res.e) {
        set_error("expansion: tracked energy disagrees with the recomputed energy");
        return IVDE_EINVAL;
    }
    std::copy(res.d.begin(), res.d.end(), labels);
    if (energy_out) *energy_out = res.e;
    if (cycles_out) *cycles_out = res.cycles;
    return IVDE_OK;
}

ivde_status ivde_optimize(const ivde_energy *energy, int32_t n_threads, int32_t partition, int32_t max_cycles,
                          int32_t *labels_out, int64_t *energy_out)
{
    Model M;
    ivde_status st = build_model(energy, M);
    if (st != IVDE_OK) return st;
    if (!labels_out || n_threads < 1 || n_threads > 4096 || max_cycles < 1 ||
        (partition != IVDE_PARTITION_BLOCKS && partition != IVDE_PARTITION_INTERLEAVED)) {
        set_error("optimize: labels_out, 1..4096 threads, a partition and max_cycles >= 1 are required");
        return IVDE_EINVAL;
    }
    const auto subs = partition_labels(M.L, n_threads, partition);
    std::vector<Result> res(subs.size());
    std::vector<uint8_t> nonsub(subs.size(), 0);
    {
        std::vector<std::thread> pool;
        for (size_t k = 0; k < subs.size(); ++k)
            pool.emplace_back([&, k] {
                bool ns = false;
                res[k].labels = subs[k];
                initial(M, subs[k], res[k].d);
                expansion(M, res[k], subs[k], max_cycles, nullptr, nullptr, ns);
                nonsub[k] = ns;
            });
        for (auto &t : pool) t.join();
    }
    for (size_t step = 1; step < res.size(); step *= 2) {
        std::vector<std::thread> pool;
        for (size_t k = 0; k + step < res.size(); k += 2 * step)
            pool.emplace_back([&, k, step] {
                bool ns = false;
                res[k] = merge(M, res[k], res[k + step], max_cycles, ns);
                nonsub[k] |= ns;
            });
        for (auto &t : pool) t.join();
    }
    for (uint8_t ns : nonsub)
        if (ns) {
            set_error("optimize: a move was not submodular (negative adjacency weight or positive reward)");
            return IVDE_EINVAL;
        }
    if (M.energy(res[0].d) != res[0].e) {
        set_error("optimize: tracked energy disagrees with the recomputed energy");
        return IVDE_EINVAL;
    }
    std::copy(res[0].d.begin(), res[0].d.end(), labels_out);
    if (energy_out) *energy_out = res[0].e;
    return IVDE_OK;
}

}  // extern "C"
