"""Oracle of the depth optimisation: Eq. (1) minimised by alpha-expansion
graph cuts over segment nodes (Sec. III-B), with the label-partitioned
threads and pairwise merging of Sec. IV-A.

TEST INFRASTRUCTURE, like the rest of this package: plain Python, slow,
written for checking by eye.

Energy of a labelling d (one label per segment row), in integer units:

    E(d) = sum_r q(w U[r, d_r])                                 optional unary, weight w
         + sum_r sum_slot [h >= 0 and d_h = d_r] q(min(0, m - K))   Eqs. (4), (5)
               with m = m[r, slot, d_r], h = hit[r, slot, d_r]
         + sum over adjacency entries (r, t) of q(beta_rt) |d_r - d_t|   Eqs. (2), (3)

q(x) = x * quantum rounded half away from zero, in FP64.  Integer terms
make every maximum flow exact, so the canonical minimum cut below is the
same for any max-flow algorithm.

A move towards label alpha lets every switchable segment keep its label
(x = 0) or take alpha (x = 1).  Among all optimal moves the one taken sets
x_i = 1 exactly when some optimal move does (the union of optimal alpha
sets): it is the cut whose source side is the set of nodes reachable from
the source in the residual graph of a maximum flow.
"""
from __future__ import annotations

import itertools
from collections import deque

import numpy as np

BLOCKS = 0
INTERLEAVED = 1


def quantize(x, quantum):
    """x * quantum rounded half away from zero (FP64), as int64."""
    y = np.asarray(x, np.float64) * float(quantum)
    return (np.sign(y) * np.floor(np.abs(y) + 0.5)).astype(np.int64)


class Energy:
    """Eq. (1) over `rows` segment nodes and `num_labels` depth levels.

    unary  [rows, L] float or None
    m, hit [rows, 2, L] (float, int) or None: the window core and the hit
           segment's row towards the two neighbouring views (Eq. (4))
    K      the truncation of Eq. (5)
    offsets, index, beta: adjacency CSR and the Eq. (3) weights, or None
    fixed  [rows] int: a label for segments that are not nodes (Sec. III-E),
           -1 for free segments, or None
    """

    def __init__(self, rows, num_labels, unary=None, m=None, hit=None, K=30.0, offsets=None, index=None,
                 beta=None, quantum=1024.0, fixed=None, unary_weight=1.0):
        self.rows, self.L = int(rows), int(num_labels)
        if unary is not None:
            self.U = quantize(float(unary_weight) * np.asarray(unary, np.float32).astype(np.float64), quantum)
        else:
            self.U = np.zeros((self.rows, self.L), np.int64)
        if m is not None:
            m64 = np.asarray(m, np.float32).astype(np.float64)
            self.hit = np.asarray(hit, np.int64)
            reward = quantize(np.minimum(0.0, m64 - float(np.float32(K))), quantum)
            self.R = np.where(self.hit >= 0, reward, 0)
        else:
            self.hit = np.full((self.rows, 2, self.L), -1, np.int64)
            self.R = np.zeros((self.rows, 2, self.L), np.int64)
        if offsets is not None:
            off = np.asarray(offsets, np.int64)
            self.er = np.repeat(np.arange(self.rows), np.diff(off))
            self.et = np.asarray(index, np.int64)
            self.ew = quantize(np.asarray(beta, np.float32), quantum)
        else:
            self.er = self.et = self.ew = np.zeros(0, np.int64)
        self.fixed = np.full(self.rows, -1, np.int64) if fixed is None else np.asarray(fixed, np.int64)

    # ------------------------------------------------------------ the energy
    def energy(self, d):
        d = np.asarray(d, np.int64)
        r = np.arange(self.rows)
        e = int(self.U[r, d].sum())
        for slot in range(2):
            h = self.hit[r, slot, d]
            ok = h >= 0
            e += int(self.R[r[ok], slot, d[ok]][d[h[ok]] == d[ok]].sum())
        e += int((self.ew * np.abs(d[self.er] - d[self.et])).sum())
        return e

    # ------------------------------------------------------------ one move
    def move_tables(self, d, alpha, switch):
        """The binary energy of the move: constant, unary tables {i: [e0, e1]}
        and pairwise tables [(i, j, [[e00, e01], [e10, e11]])] over the
        switchable segments (switch[i] True), each term evaluated from its
        definition at the labels the two choices give."""
        d = np.asarray(d, np.int64)

        def lab(i, x):
            return alpha if (x and switch[i]) else int(d[i])

        const = 0
        unary = {}
        pair = []

        def add(vars_, f):
            nonlocal const
            sv = [v for v in vars_ if switch[v]]
            if not sv:
                const += f({v: 0 for v in vars_})
            elif len(set(sv)) == 1:
                i = sv[0]
                t = unary.setdefault(i, [0, 0])
                for x in (0, 1):
                    t[x] += f({v: x if v == i else 0 for v in vars_})
            else:
                i, j = sv[0], sv[1]
                tab = [[0, 0], [0, 0]]
                for xi in (0, 1):
                    for xj in (0, 1):
                        tab[xi][xj] = f({v: (xi if v == i else xj if v == j else 0) for v in vars_})
                pair.append((i, j, tab))

        for r in range(self.rows):
            add([r], lambda x, r=r: int(self.U[r, lab(r, x[r])]))
            for slot in range(2):
                # candidate labels of r in this move: its own, and alpha if switchable
                for xr in ((0, 1) if switch[r] else (0,)):
                    c = lab(r, xr)
                    h = int(self.hit[r, slot, c])
                    if h < 0:
                        continue
                    R = int(self.R[r, slot, c])
                    # [label_r = c][label_h = c] R
                    vs = [r, h] if h != r else [r]
                    add(vs, lambda x, r=r, h=h, c=c, R=R: R * int(lab(r, x[r]) == c and lab(h, x[h]) == c))
        for k in range(len(self.er)):
            r, t, w = int(self.er[k]), int(self.et[k]), int(self.ew[k])
            add([r, t], lambda x, r=r, t=t, w=w: w * abs(lab(r, x[r]) - lab(t, x[t])))
        return const, unary, pair

    def best_move(self, d, alpha, switch, brute_limit=0):
        """The canonical optimal move: x [rows] of 0/1 (0 for segments that
        cannot switch).  brute_limit > 0 enumerates all moves when at most
        that many segments can switch; otherwise max-flow."""
        const, unary, pair = self.move_tables(d, alpha, switch)
        nodes = [i for i in range(self.rows) if switch[i]]
        if brute_limit and len(nodes) <= brute_limit:
            return self._brute_move(nodes, const, unary, pair)
        return self._cut_move(nodes, unary, pair)

    @staticmethod
    def _binary_value(x, const, unary, pair):
        e = const
        for i, t in unary.items():
            e += t[x[i]]
        for i, j, tab in pair:
            e += tab[x[i]][x[j]]
        return e

    def _brute_move(self, nodes, const, unary, pair):
        best, union = None, np.zeros(self.rows, np.int64)
        x = np.zeros(self.rows, np.int64)
        for bits in itertools.product((0, 1), repeat=len(nodes)):
            x[nodes] = bits
            e = self._binary_value(x, const, unary, pair)
            if best is None or e < best:
                best, union = e, x.copy()
            elif e == best:
                union |= x
        return union

    def _cut_move(self, nodes, unary, pair):
        """Kolmogorov-Zabih graph: x_i = 0 on the source side.  A unary
        [e0, e1] adds e1 - e0 to source->i (cut when x_i = 1) if positive,
        else e0 - e1 to i->sink; a pair table [[A, B], [C, D]] is
        A + (C - A) x_i + (D - C) x_j + (B + C - A - D)(1 - x_i) x_j, the last
        an edge i->j of capacity B + C - A - D (>= 0 for these moves)."""
        S, T = "s", "t"
        cap = {}

        def addc(u, v, c):
            if c:
                cap[(u, v)] = cap.get((u, v), 0) + c
                cap.setdefault((v, u), 0)

        tl = {i: 0 for i in nodes}           # net unary: cost of x_i = 1 minus cost of x_i = 0
        for i, t in unary.items():
            tl[i] += t[1] - t[0]
        for i, j, tab in pair:
            (A, B), (C, D) = tab
            w = B + C - A - D
            if w < 0:
                raise ValueError("non-submodular pair term in a move")
            tl[i] += C - A
            tl[j] += D - C
            addc(i, j, w)
        for i in nodes:
            if tl[i] > 0:
                addc(S, i, tl[i])
            elif tl[i] < 0:
                addc(i, T, -tl[i])
        adj = {}
        for (u, v) in cap:
            adj.setdefault(u, []).append(v)
        max_flow_edmonds_karp(cap, adj, S, T)
        # source side: reachable from s in the residual graph
        seen = {S}
        q = deque([S])
        while q:
            u = q.popleft()
            for v in adj.get(u, []):
                if v not in seen and cap[(u, v)] > 0:
                    seen.add(v)
                    q.append(v)
        x = np.zeros(self.rows, np.int64)
        for i in nodes:
            x[i] = 0 if i in seen else 1
        return x

    # ------------------------------------------------------------ expansion
    def switchable(self, d, alpha, allowed=None):
        d = np.asarray(d)
        sw = (self.fixed < 0) & (d != alpha)
        if allowed is not None:
            sw &= np.array([alpha in a for a in allowed])
        return sw

    def expansion(self, d0, labels, allowed=None, max_cycles=8, brute_limit=0):
        """Alpha-expansion: cycles over `labels` in increasing order; a move
        is taken when it lowers the energy; stops after a cycle without a
        change or after max_cycles.  Returns (labelling, energy, cycles)."""
        d = np.asarray(d0, np.int64).copy()
        e = self.energy(d)
        cycles = 0
        for _ in range(max_cycles):
            cycles += 1
            changed = False
            for alpha in sorted(labels):
                sw = self.switchable(d, alpha, allowed)
                if not sw.any():
                    continue
                x = self.best_move(d, alpha, sw, brute_limit)
                d2 = np.where(x == 1, alpha, d)
                e2 = self.energy(d2)
                if e2 < e:
                    d, e, changed = d2, e2, True
            if not changed:
                break
        return d, e, cycles

    # ------------------------------------------------------------ Sec. IV-A
    def initial(self, labels):
        """Each free segment starts at the label of the subset with the
        lowest unary cost (lowest label on ties); fixed segments at theirs."""
        labels = np.array(sorted(labels))
        d = labels[np.argmin(self.U[:, labels], axis=1)]
        return np.where(self.fixed >= 0, self.fixed, d)

    def optimize(self, n_threads=1, partition=BLOCKS, max_cycles=8, brute_limit=0):
        """Label-partitioned estimation: thread k expands over its subset of
        labels; results merge pairwise (k with k + 2^c in cycle c), each merge
        an expansion over both subsets in which a segment may only take one
        of its two candidate labels.  Returns (labelling, energy)."""
        subsets = partition_labels(self.L, n_threads, partition)
        res = []
        for sub in subsets:
            d, e, _ = self.expansion(self.initial(sub), sub, None, max_cycles, brute_limit)
            res.append((d, e, sorted(sub)))
        step = 1
        while step < len(res):
            for k in range(0, len(res), 2 * step):
                if k + step < len(res):
                    res[k] = self.merge(res[k], res[k + step], max_cycles, brute_limit)
            step *= 2
        return res[0][0], res[0][1]

    def merge(self, A, B, max_cycles=8, brute_limit=0):
        """Merge two labellings: start from the one with the lower energy
        (the first on a tie), expand over the union of both label sets, each
        segment restricted to its two candidate labels."""
        (da, ea, la), (db, eb, lb) = A, B
        start = da if ea <= eb else db
        allowed = [{int(a), int(b)} for a, b in zip(da, db)]
        labels = sorted(set(la) | set(lb))
        d, e, _ = self.expansion(start, labels, allowed, max_cycles, brute_limit)
        return d, e, labels


def partition_labels(L, n, partition):
    """Sec. IV-A: n subsets of the L levels, as blocks (subset k holds
    [floor(k L / n), floor((k + 1) L / n))) or interleaved (l mod n = k);
    empty subsets are dropped."""
    n = max(1, min(int(n), int(L)))
    if partition == BLOCKS:
        subs = [list(range(k * L // n, (k + 1) * L // n)) for k in range(n)]
    else:
        subs = [list(range(k, L, n)) for k in range(n)]
    return [s for s in subs if s]


def max_flow_edmonds_karp(cap, adj, s, t):
    """Edmonds-Karp: augment along shortest residual paths until none is
    left; `cap` is updated in place to the residual capacities."""
    flow = 0
    while True:
        parent = {s: None}
        q = deque([s])
        while q and t not in parent:
            u = q.popleft()
            for v in adj.get(u, []):
                if v not in parent and cap[(u, v)] > 0:
                    parent[v] = u
                    q.append(v)
        if t not in parent:
            return flow
        b, v = None, t
        while parent[v] is not None:
            u = parent[v]
            b = cap[(u, v)] if b is None else min(b, cap[(u, v)])
            v = u
        v = t
        while parent[v] is not None:
            u = parent[v]
            cap[(u, v)] -= b
            cap[(v, u)] += b
            v = u
        flow += b


def min_cut_brute(n, cap_edges, s, t):
    """Minimum s-t cut of a graph on nodes 0..n-1 by enumeration: returns
    (value, union of the sink sides of all minimum cuts)."""
    best, union = None, set()
    others = [v for v in range(n) if v not in (s, t)]
    for bits in itertools.product((0, 1), repeat=len(others)):
        sink = {t} | {v for v, b in zip(others, bits) if b}
        val = sum(c for (u, v), c in cap_edges.items() if u not in sink and v in sink)
        if best is None or val < best:
            best, union = val, set(sink)
        elif val == best:
            union |= sink
    return best, union
