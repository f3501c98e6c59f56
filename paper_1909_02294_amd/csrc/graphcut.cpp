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
        first_.assign(n, -1);
        tr_.assign(n, 0);
        head_.clear();
        next_.clear();
        rcap_.clear();
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
    void add_edge(int i, int j, int64_t c)
    {
        const int a = (int)head_.size();
        head_.push_back(j);
        next_.push_back(first_[i]);
        rcap_.push_back(c);
        first_[i] = a;
        head_.push_back(i);
        next_.push_back(first_[j]);
        rcap_.push_back(0);
        first_[j] = a + 1;
    }
    int64_t solve();
    // nodes reachable from the source in the residual graph
    void source_side(std::vector<uint8_t> &out) const;

private:
    static constexpr int kTerminal = -2, kOrphan = -3, kNone = -1;
    static int sister(int a) { return a ^ 1; }
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
    std::vector<int> first_, head_, next_;
    std::vector<int64_t> rcap_, tr_;
    int64_t flow_ = 0;
    // search state
    std::vector<int> parent_, ts_, dist_;
    std::vector<uint8_t> sink_, queued_;
    std::vector<int> queue_, orphans_;
    size_t qhead_ = 0;
    int time_ = 0;
};

int64_t MaxFlow::solve()
{
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
        if (tr_[i] > 0) {
            parent_[i] = kTerminal;
            sink_[i] = 0;
            dist_[i] = 1;
            set_active(i);
        } else if (tr_[i] < 0) {
            parent_[i] = kTerminal;
            sink_[i] = 1;
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
        if (!sink_[i]) {
            for (int a = first_[i]; a >= 0; a = next_[a]) {
                if (rcap_[a] <= 0) continue;
                const int j = head_[a];
                if (parent_[j] == kNone) {
                    sink_[j] = 0;
                    parent_[j] = sister(a);
                    ts_[j] = ts_[i];
                    dist_[j] = dist_[i] + 1;
                    set_active(j);
                } else if (sink_[j]) {
                    mid = a;
                    break;
                } else if (ts_[j] <= ts_[i] && dist_[j] > dist_[i]) {
                    parent_[j] = sister(a);
                    ts_[j] = ts_[i];
                    dist_[j] = dist_[i] + 1;
                }
            }
        } else {
            for (int a = first_[i]; a >= 0; a = next_[a]) {
                if (rcap_[sister(a)] <= 0) continue;
                const int j = head_[a];
                if (parent_[j] == kNone) {
                    sink_[j] = 1;
                    parent_[j] = sister(a);
                    ts_[j] = ts_[i];
                    dist_[j] = dist_[i] + 1;
                    set_active(j);
                } else if (!sink_[j]) {
                    mid = sister(a);
                    break;
                } else if (ts_[j] <= ts_[i] && dist_[j] > dist_[i]) {
                    parent_[j] = sister(a);
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
void MaxFlow::augment(int mid)
{
    int64_t b = rcap_[mid];
    int i;
    for (i = head_[sister(mid)];; i = head_[parent_[i]]) {
        const int a = parent_[i];
        if (a == kTerminal) break;
        b = std::min(b, rcap_[sister(a)]);
    }
    b = std::min(b, tr_[i]);
    for (i = head_[mid];; i = head_[parent_[i]]) {
        const int a = parent_[i];
        if (a == kTerminal) break;
        b = std::min(b, rcap_[a]);
    }
    b = std::min(b, -tr_[i]);

    rcap_[sister(mid)] += b;
    rcap_[mid] -= b;
    for (i = head_[sister(mid)];;) {
        const int a = parent_[i];
        if (a == kTerminal) {
            tr_[i] -= b;
            if (tr_[i] == 0) {
                parent_[i] = kOrphan;
                orphans_.push_back(i);
            }
            break;
        }
        rcap_[a] += b;
        rcap_[sister(a)] -= b;
        const int up = head_[a];
        if (rcap_[sister(a)] == 0) {
            parent_[i] = kOrphan;
            orphans_.push_back(i);
        }
        i = up;
    }
    for (i = head_[mid];;) {
        const int a = parent_[i];
        if (a == kTerminal) {
            tr_[i] += b;
            if (tr_[i] == 0) {
                parent_[i] = kOrphan;
                orphans_.push_back(i);
            }
            break;
        }
        rcap_[sister(a)] += b;
        rcap_[a] -= b;
        const int down = head_[a];
        if (rcap_[a] == 0) {
            parent_[i] = kOrphan;
            orphans_.push_back(i);
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
        const int i = orphans_.back();
        orphans_.pop_back();
        const bool sink = sink_[i];
        int best = -1;
        int dmin = INT_MAX;
        for (int a0 = first_[i]; a0 >= 0; a0 = next_[a0]) {
            // residual towards i (source tree) or away from i (sink tree)
            if ((sink ? rcap_[a0] : rcap_[sister(a0)]) <= 0) continue;
            const int j = head_[a0];
            if (sink_[j] != sink || parent_[j] == kNone) continue;
            // does j's path reach the terminal?
            int d = 0;
            int k = j;
            for (;;) {
                if (ts_[k] == time_) {
                    d += dist_[k];
                    break;
                }
                const int a = parent_[k];
                ++d;
                if (a == kTerminal) {
                    ts_[k] = time_;
                    dist_[k] = 1;
                    break;
                }
                if (a == kOrphan) {
                    d = INT_MAX;
                    break;
                }
                k = head_[a];
            }
            if (d == INT_MAX) continue;
            if (d < dmin) {
                best = a0;
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
        for (int a0 = first_[i]; a0 >= 0; a0 = next_[a0]) {
            const int j = head_[a0];
            if (sink_[j] != sink || parent_[j] == kNone) continue;
            if ((sink ? rcap_[a0] : rcap_[sister(a0)]) > 0) set_active(j);
            const int a = parent_[j];
            if (a != kTerminal && a != kOrphan && head_[a] == i) {
                parent_[j] = kOrphan;
                orphans_.insert(orphans_.begin(), j);
            }
        }
        parent_[i] = kNone;
    }
}

void MaxFlow::source_side(std::vector<uint8_t> &out) const
{
    out.assign(n_, 0);
    std::vector<int> st;
    for (int i = 0; i < n_; ++i)
        if (tr_[i] > 0) {
            out[i] = 1;
            st.push_back(i);
        }
    while (!st.empty()) {
        const int i = st.back();
        st.pop_back();
        for (int a = first_[i]; a >= 0; a = next_[a]) {
            const int j = head_[a];
            if (!out[j] && rcap_[a] > 0) {
                out[j] = 1;
                st.push_back(j);
            }
        }
    }
}

// ------------------------------------------------------------------ energy
int64_t quantize(double x, double q) { return (int64_t)std::llround(x * q); }

struct Model {
    int64_t rows = 0;
    int L = 0;
    std::vector<int64_t> U;          // [rows][L] or empty
    std::vector<int64_t> R;          // [rows][2][L] rewards, 0 without a hit, or empty
    const int32_t *hit = nullptr;    // [rows][2][L]
    const int64_t *off = nullptr;
    const int32_t *idx = nullptr;
    std::vector<int64_t> W;          // per adjacency entry
    std::vector<int32_t> fixed;      // label or -1

    int64_t unary(int64_t r, int l) const { return U.empty() ? 0 : U[r * L + l]; }
    int32_t hit_at(int64_t r, int s, int l) const { return hit ? hit[(r * 2 + s) * L + l] : -1; }
    int64_t reward(int64_t r, int s, int l) const { return R.empty() ? 0 : R[(r * 2 + s) * L + l]; }

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
            if (off)
                for (int64_t k = off[r]; k < off[r + 1]; ++k) e += W[k] * std::abs(l - d[idx[k]]);
        }
        return e;
    }
};

// One alpha-expansion move over the segments allowed to switch.
class Mover {
public:
    explicit Mover(const Model &m) : M(m), node_(m.rows, -1) {}

    // Returns true (and updates d, e) when the canonical optimal move lowers the energy.
    bool move(std::vector<int32_t> &d, int64_t &e, int alpha, const std::vector<int32_t> *cand_a,
              const std::vector<int32_t> *cand_b)
    {
        // switchable segments: free, not at alpha, and (in a merge) alpha among their candidates
        nodes_.clear();
        for (int64_t r = 0; r < M.rows; ++r) {
            bool sw = M.fixed.empty() || M.fixed[r] < 0;
            sw = sw && d[r] != alpha;
            if (sw && cand_a) sw = (*cand_a)[r] == alpha || (*cand_b)[r] == alpha;
            node_[r] = sw ? (int)nodes_.size() : -1;
            if (sw) nodes_.push_back(r);
        }
        if (nodes_.empty()) return false;
        const int n = (int)nodes_.size();
        g_.reset(n);
        net_.assign(n, 0);
        auto lab = [&](int64_t r, int x) { return (x && node_[r] >= 0) ? alpha : d[r]; };
        auto unary1 = [&](int i, int64_t c0, int64_t c1) { net_[i] += c1 - c0; };
        auto pair = [&](int i, int j, int64_t A, int64_t B, int64_t C, int64_t D) {
            // A + (C - A) x_i + (D - C) x_j + (B + C - A - D)(1 - x_i) x_j
            net_[i] += C - A;
            net_[j] += D - C;
            const int64_t w = B + C - A - D;
            if (w > 0) g_.add_edge(i, j, w);
            if (w < 0) nonsub_ = true;
        };
        nonsub_ = false;
        for (int64_t r = 0; r < M.rows; ++r) {
            const int ir = node_[r];
            if (ir >= 0) unary1(ir, M.unary(r, d[r]), M.unary(r, alpha));
            for (int s = 0; s < 2; ++s) {
                for (int xr = 0; xr < (ir >= 0 ? 2 : 1); ++xr) {
                    const int c = lab(r, xr);
                    const int32_t h = M.hit_at(r, s, c);
                    if (h < 0) continue;
                    const int64_t Rv = M.reward(r, s, c);
                    if (Rv == 0) continue;
                    const int ih = node_[h];
                    // Rv [label_r = c][label_h = c]
                    if (h == r) {
                        if (ir >= 0) unary1(ir, xr == 0 ? Rv : 0, xr == 1 ? Rv : 0);
                    } else if (ir >= 0 && ih >= 0) {
                        int64_t t[2][2];
                        for (int a = 0; a < 2; ++a)
                            for (int b = 0; b < 2; ++b) t[a][b] = (a == xr && lab(h, b) == c) ? Rv : 0;
                        pair(ir, ih, t[0][0], t[0][1], t[1][0], t[1][1]);
                    } else if (ir >= 0) {
                        const int64_t v = d[h] == c ? Rv : 0;
                        unary1(ir, xr == 0 ? v : 0, xr == 1 ? v : 0);
                    } else if (ih >= 0) {
                        unary1(ih, lab(h, 0) == c ? Rv : 0, lab(h, 1) == c ? Rv : 0);
                    }
                }
            }
            if (M.off) {
                for (int64_t k = M.off[r]; k < M.off[r + 1]; ++k) {
                    const int64_t t = M.idx[k];
                    const int it = node_[t];
                    const int64_t w = M.W[k];
                    if (w == 0 || (ir < 0 && it < 0)) continue;
                    if (ir >= 0 && it >= 0) {
                        pair(ir, it, w * std::abs(d[r] - d[t]), w * std::abs(d[r] - alpha),
                             w * std::abs(alpha - d[t]), 0);
                    } else if (ir >= 0) {
                        unary1(ir, w * std::abs(d[r] - d[t]), w * std::abs(alpha - d[t]));
                    } else {
                        unary1(it, w * std::abs(d[r] - d[t]), w * std::abs(d[r] - alpha));
                    }
                }
            }
        }
        for (int i = 0; i < n; ++i) {
            if (net_[i] > 0)
                g_.add_tweights(i, net_[i], 0);
            else if (net_[i] < 0)
                g_.add_tweights(i, 0, -net_[i]);
        }
        g_.solve();
        g_.source_side(side_);
        cand_ = d;
        bool any = false;
        for (int i = 0; i < n; ++i)
            if (!side_[i]) {
                cand_[nodes_[i]] = alpha;
                any = true;
            }
        if (!any) return false;
        const int64_t e2 = M.energy(cand_);
        if (e2 >= e) return false;
        d.swap(cand_);
        e = e2;
        return true;
    }

    bool nonsubmodular() const { return nonsub_; }

private:
    const Model &M;
    std::vector<int> node_;
    std::vector<int64_t> nodes_;
    std::vector<int64_t> net_;
    std::vector<uint8_t> side_;
    std::vector<int32_t> cand_;
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
    res.e = M.energy(res.d);
    res.cycles = 0;
    for (int c = 0; c < max_cycles; ++c) {
        ++res.cycles;
        bool changed = false;
        for (int alpha : labels) changed |= mv.move(res.d, res.e, alpha, cand_a, cand_b);
        nonsub |= mv.nonsubmodular();
        if (!changed) break;
    }
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
    for (int64_t r = 0; r < M.rows; ++r) {
        if (!M.fixed.empty() && M.fixed[r] >= 0) {
            d[r] = M.fixed[r];
            continue;
        }
        int best = labels[0];
        int64_t bv = M.unary(r, best);
        for (int l : labels)
            if (M.unary(r, l) < bv) {
                bv = M.unary(r, l);
                best = l;
            }
        d[r] = best;
    }
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
    if (E->unary) {
        if (!std::isfinite(E->unary_weight)) {
            set_error("energy: unary_weight must be finite");
            return IVDE_EINVAL;
        }
        M.U.resize((size_t)rows * L);
        for (size_t i = 0; i < M.U.size(); ++i) {
            const double u = E->unary_weight * (double)E->unary[i];
            if (!(std::fabs(u * q) < limit)) {
                set_error("energy: unary value %g too large for quantum %g", u, q);
                return IVDE_EINVAL;
            }
            M.U[i] = quantize(u, q);
        }
    }
    if (E->window_m) {
        M.hit = E->window_hit;
        M.R.resize((size_t)rows * 2 * L);
        for (size_t i = 0; i < M.R.size(); ++i) {
            const int32_t h = E->window_hit[i];
            if (h < -1 || h >= rows) {
                set_error("energy: window_hit entry %zu (%d) outside [-1, rows)", i, h);
                return IVDE_EINVAL;
            }
            if (h < 0) {
                M.R[i] = 0;
                continue;
            }
            const double v = std::min(0.0, (double)E->window_m[i] - (double)E->K);
            if (!(std::fabs(v * q) < limit)) {
                set_error("energy: window value %g too large for quantum %g", (double)E->window_m[i], q);
                return IVDE_EINVAL;
            }
            M.R[i] = quantize(v, q);
        }
    }
    if (E->adj_offsets) {
        M.off = E->adj_offsets;
        M.idx = E->adj_index;
        if (M.off[0] != 0) {
            set_error("energy: adjacency offsets must start at 0");
            return IVDE_EINVAL;
        }
        for (int64_t r = 0; r < rows; ++r)
            if (M.off[r + 1] < M.off[r]) {
                set_error("energy: adjacency offsets decrease at row %lld", (long long)r);
                return IVDE_EINVAL;
            }
        const int64_t n = M.off[rows];
        M.W.resize((size_t)n);
        for (int64_t k = 0; k < n; ++k) {
            if (M.idx[k] < 0 || M.idx[k] >= rows) {
                set_error("energy: adjacency entry %lld names row %d", (long long)k, M.idx[k]);
                return IVDE_EINVAL;
            }
            const double v = (double)E->adj_beta[k] * q;
            if (!(E->adj_beta[k] >= 0.f) || !(v < limit / L)) {
                set_error("energy: beta %g must be >= 0 and small enough for quantum %g", (double)E->adj_beta[k], q);
                return IVDE_EINVAL;
            }
            M.W[k] = quantize(E->adj_beta[k], q);
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
    std::copy(res[0].d.begin(), res[0].d.end(), labels_out);
    if (energy_out) *energy_out = res[0].e;
    return IVDE_OK;
}

}  // extern "C"
