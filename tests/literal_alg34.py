"""A second, literal reading of the paper's parallel GOMEA for tiny graphs (test-only).

It follows the structure of Algorithm 3 and Algorithm 4 as printed, with whole-population
arrays: a copy O' receives every donor insertion of a group (DetermineAndInsertDonorGenes);
the dependent subfunctions of every set of the group are listed with their set as key, all
of them are evaluated on O and on O', summed per (set, solution) key with a reduce-by-key
(numpy's add.at), and subtracted to give the delta matrix; the improvement mask M_IMP then
decides which steps are kept (ResetNonImprovements / InsertImprovements).  The C oracle
instead applies one step at a time.  Both must agree exactly.

Random draws use the oracle's Philox4x32-10 (itself pinned against numpy's Philox) with the
same counters: class order (g, 0xFFFFFFFF, t, 0), donor field (g, c, i, p // 8).
"""
from __future__ import annotations

import numpy as np

import oracle


def _draw(seed, c0, c1, c2, c3):
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    return oracle.philox4x32(key, [c0 & 0xFFFFFFFF, c1 & 0xFFFFFFFF, c2, c3])


def initial_population(n, N, seed):
    """InitializePopulation: gene v of solution i = bit (v mod 32) of word ((v / 32) mod 4) of
    Philox(seed; 0xFFFFFFFF, i, v / 128, 0)."""
    P = np.zeros((N, n), np.uint8)
    for i in range(N):
        for blk in range((n + 127) // 128):
            out = _draw(seed, 0xFFFFFFFF, i, blk, 0)
            for v in range(blk * 128, min(n, blk * 128 + 128)):
                P[i, v] = (int(out[(v >> 5) & 3]) >> (v & 31)) & 1
    return P


class LiteralParGomea:
    def __init__(self, g, set_ptr, set_vars, classes, N, seed, rule=0, order=0, P=None,
                 fi=False, fi_stop_on_accept=False):
        self.fi = fi
        self.fi_stop_on_accept = fi_stop_on_accept  # a wrong reading, kept to find cases
        # where it differs from the paper's (stop at the first step that raises fitness)
        self.g = g
        self.sets = [np.asarray(set_vars[set_ptr[j]:set_ptr[j + 1]]) for j in
                     range(len(set_ptr) - 1)]
        self.classes = classes                      # list of lists of set indices (ascending)
        if P is None:
            P = initial_population(g.n, N, seed)
        self.P = np.array(P, dtype=np.uint8)        # N x n
        self.N, self.n = self.P.shape
        self.seed, self.rule, self.order = seed, rule, order
        self.f = np.array([self.fitness(x) for x in self.P], dtype=np.int64)
        b = int(np.argmax(self.f))                  # first maximum = lowest index
        self.E, self.fE = self.P[b].copy(), int(self.f[b])
        self.gen = 0
        self.evaluated = 0
        self.accepted = 0
        # incident edges per vertex = DependentSubfunctions(u) for Max-Cut
        self.inc = [[] for _ in range(self.n)]
        for e in range(g.m):
            self.inc[g.u[e]].append(e)
            self.inc[g.v[e]].append(e)

    def fitness(self, x):
        # Max-Cut, Section 6.2, with x in {-1, 1}: one half of sum w (1 - x_u x_v)
        s = 2 * x.astype(np.int64) - 1
        return int(np.sum(self.g.w.astype(np.int64) * (1 - s[self.g.u] * s[self.g.v])) // 2)

    def group_order(self):
        k = len(self.classes)
        perm = list(range(k))
        if self.order == 0:
            for t in range(k - 1, 0, -1):
                r = int((int(_draw(self.seed, self.gen, 0xFFFFFFFF, t, 0)[0]) * (t + 1)) >> 32)
                perm[t], perm[r] = perm[r], perm[t]
        return perm

    def generation(self, stop_after=None):
        """One generation.  With stop_after = t, a copy of (O, f, evaluated, accepted) taken
        right after the group at order position t is kept in self.mid."""
        N, g = self.N, self.g
        eq = np.array([np.array_equal(self.P[i], self.E) for i in range(N)])
        O = self.P.copy()                                        # Clone(P)
        improved_any = np.zeros(N, dtype=bool)
        order = self.group_order()
        for t, c in enumerate(order):
            G = self.classes[c]
            # DetermineAndInsertDonorGenes
            Op = O.copy()
            has = np.zeros((len(G), N), dtype=bool)
            for p, j in enumerate(G):
                F = self.sets[j]
                for i in range(N):
                    D = [d for d in range(N) if d != i and np.any(self.P[d, F] != O[i, F])]
                    if not D:
                        continue
                    out = _draw(self.seed, self.gen, c, i, p >> 3)
                    h = (int(out[(p & 7) >> 1]) >> (16 * (p & 1))) & 0xFFFF
                    d = D[(h * len(D)) >> 16]
                    Op[i, F] = self.P[d, F]
                    has[p, i] = True
            # ParallelPartialEvaluations (Algorithm 4)
            Fdep, Kdep = [], []
            for p, j in enumerate(G):
                deps = sorted({e for u in self.sets[j] for e in self.inc[u]})
                Fdep += deps
                Kdep += [p] * len(deps)
            Fdep, Kdep = np.asarray(Fdep, np.int64), np.asarray(Kdep, np.int64)
            stride = max(len(Kdep), len(G))
            keys = Kdep[:, None] + np.arange(N)[None, :] * stride            # M_dep[u, v]
            w = g.w.astype(np.int64)[Fdep][:, None]
            FO = w * (O[:, g.u[Fdep]] != O[:, g.v[Fdep]]).T                   # on O
            FOp = w * (Op[:, g.u[Fdep]] != Op[:, g.v[Fdep]]).T                # on O'
            outO = np.zeros(stride * N, np.int64)
            outOp = np.zeros(stride * N, np.int64)
            np.add.at(outO, keys.ravel(), FO.ravel())                         # ReduceByKey
            np.add.at(outOp, keys.ravel(), FOp.ravel())
            idx = np.arange(len(G))[:, None] + np.arange(N)[None, :] * stride
            delta = outOp[idx] - outO[idx]                                    # |G| x N
            # DetermineImprovements
            neutral = (self.rule == 1) | ~eq[None, :]
            M = has & ((delta > 0) | ((delta == 0) & neutral))
            # ResetNonImprovements + InsertImprovements
            for p, j in enumerate(G):
                F = self.sets[j]
                for i in range(N):
                    if M[p, i]:
                        O[i, F] = Op[i, F]
                        self.f[i] += delta[p, i]
            self.evaluated += int(has.sum())
            self.accepted += int(M.sum())
            improved_any |= M.any(axis=0)
            if t == stop_after:
                self.mid = (O.copy(), self.f.copy(), self.evaluated, self.accepted)
        if self.fi:
            self.forced_improvement(O, eq, improved_any, order)
        self.P = O                                               # P <- O
        b = int(np.argmax(self.f))
        if self.f[b] > self.fE:
            self.E, self.fE = self.P[b].copy(), int(self.f[b])
        self.gen += 1

    def forced_improvement(self, O, eq, improved_any, order):
        """ApplyForcedImprovement as the paper describes the serial procedure (Section 4): a
        solution with no accepted variation in this generation undergoes GOM with the
        elitist as donor, set after set (here in the generation's group order, sets of a
        group ascending); the first step that raises its fitness ends the procedure; if none
        does, a copy of the elitist takes its place."""
        for i in range(self.N):
            if improved_any[i]:
                continue
            done = False
            for c in order:
                for j in self.classes[c]:
                    F = self.sets[j]
                    if np.array_equal(O[i, F], self.E[F]):
                        continue
                    self.evaluated += 1
                    trial = O[i].copy()
                    trial[F] = self.E[F]
                    delta = self.fitness(trial) - self.fitness(O[i])
                    if delta > 0 or (delta == 0 and (self.rule == 1 or not eq[i])):
                        O[i] = trial
                        self.f[i] += delta
                        self.accepted += 1
                    if delta > 0 or (self.fi_stop_on_accept and delta == 0 and
                                     (self.rule == 1 or not eq[i])):
                        done = True
                        break
                if done:
                    break
            if not done:
                O[i] = self.E
                self.f[i] = self.fE
