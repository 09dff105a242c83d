"""An independent whole-population reference of parallel GOM for tiny graphs (test-only).

Written from the definitions rather than from any printed procedure:

* a colour class is a set of mutually independent FOS sets (Section 5.1), so every
  (solution, set) pair of the class may be decided against the offspring as it stood when the
  class began, and all accepted changes then applied together;
* the value of a trial solution is the Max-Cut objective itself (Section 6.2), evaluated in
  full on the trial and on the current offspring; no partial evaluation is used, so a mistake
  in the oracle's delta (a dropped edge, a wrong sign, an edge counted twice) shows up here;
* the donor rule (Section 4: a uniformly drawn population member that differs from the
  offspring on the set), the acceptance rule (Section 5.3: better, or equal while the
  solution at the generation start differs from the elitist) and the elitist update at the
  generation end.

The C oracle instead applies one step after another inside a class with partial deltas.  Both
must agree exactly, every generation.

Random draws use the oracle's Philox4x32-10 (pinned by published known answers) with the same
counters as the method's reading: class order (g, 0xFFFFFFFF, t, 0), donor field
(g, c, i, p // 8), initial genes (0xFFFFFFFF, i, v // 128, 0).
"""
from __future__ import annotations

import numpy as np

import oracle


def _draw(seed, c0, c1, c2, c3):
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    return oracle.philox4x32(key, [c0 & 0xFFFFFFFF, c1 & 0xFFFFFFFF, c2, c3])


def initial_population(n, N, seed):
    """Uniform random genes: gene v of solution i = bit (v mod 32) of word ((v / 32) mod 4) of
    Philox(seed; 0xFFFFFFFF, i, v / 128, 0)."""
    P = np.zeros((N, n), np.uint8)
    for i in range(N):
        for blk in range((n + 127) // 128):
            out = _draw(seed, 0xFFFFFFFF, i, blk, 0)
            for v in range(blk * 128, min(n, blk * 128 + 128)):
                P[i, v] = (int(out[(v >> 5) & 3]) >> (v & 31)) & 1
    return P


class ClassAtOnceGomea:
    """Parallel GOM with every colour class decided at once and objectives evaluated in full."""

    def __init__(self, g, set_ptr, set_vars, classes, N, seed, rule=0, order=0, P=None,
                 fi=False, fi_stop_on_accept=False):
        self.fi = fi
        # A deliberately wrong reading of forced improvement (stop at the first accepted step
        # rather than the first improving one), kept to show that the two readings differ.
        self.fi_stop_on_accept = fi_stop_on_accept
        self.g = g
        self.sets = [np.asarray(set_vars[set_ptr[j]:set_ptr[j + 1]]) for j in
                     range(len(set_ptr) - 1)]
        self.classes = classes                      # list of lists of set indices (ascending)
        if P is None:
            P = initial_population(g.n, N, seed)
        self.P = np.array(P, dtype=np.uint8)        # N x n, generation-start population
        self.N, self.n = self.P.shape
        self.seed, self.rule, self.order = seed, rule, order
        self.f = np.array([self.objective(x) for x in self.P], dtype=np.int64)
        b = int(np.argmax(self.f))                  # first maximum = lowest index
        self.E, self.fE = self.P[b].copy(), int(self.f[b])
        self.gen = 0
        self.evaluated = 0
        self.accepted = 0

    def objective(self, x):
        """Max-Cut with x in {-1, 1}: one half of the sum over edges of w (1 - x_u x_v)."""
        s = 2 * x.astype(np.int64) - 1
        return int(np.sum(self.g.w.astype(np.int64) * (1 - s[self.g.u] * s[self.g.v])) // 2)

    def class_order(self):
        k = len(self.classes)
        perm = list(range(k))
        if self.order == 0:
            for t in range(k - 1, 0, -1):
                r = int((int(_draw(self.seed, self.gen, 0xFFFFFFFF, t, 0)[0]) * (t + 1)) >> 32)
                perm[t], perm[r] = perm[r], perm[t]
        return perm

    def donor(self, c, i, p, F, Oi):
        """Uniform draw among the members d != i whose genes on F differ from Oi; None if none."""
        eligible = [d for d in range(self.N) if d != i and np.any(self.P[d, F] != Oi[F])]
        if not eligible:
            return None
        word = int(_draw(self.seed, self.gen, c, i, p >> 3)[(p & 7) >> 1])
        h = (word >> (16 * (p & 1))) & 0xFFFF
        return eligible[(h * len(eligible)) >> 16]

    def may_accept(self, delta, eq_i):
        return delta > 0 or (delta == 0 and (self.rule == 1 or not eq_i))

    def generation(self, stop_after=None):
        """One generation.  With stop_after = t, a copy of (O, f, evaluated, accepted) taken
        right after the class at order position t is kept in self.mid."""
        N = self.N
        eq = [bool(np.array_equal(self.P[i], self.E)) for i in range(N)]
        O = self.P.copy()
        any_accepted = np.zeros(N, dtype=bool)
        order = self.class_order()
        for t, c in enumerate(order):
            start = O.copy()            # every pair of the class sees the class-start offspring
            decisions = []
            for p, j in enumerate(self.classes[c]):
                F = self.sets[j]
                for i in range(N):
                    d = self.donor(c, i, p, F, start[i])
                    if d is None:
                        continue
                    self.evaluated += 1
                    trial = start[i].copy()
                    trial[F] = self.P[d, F]
                    delta = self.objective(trial) - self.objective(start[i])
                    if self.may_accept(delta, eq[i]):
                        decisions.append((i, F, self.P[d, F].copy(), delta))
            for i, F, genes, delta in decisions:     # sets of a class are disjoint per solution
                O[i, F] = genes
                self.f[i] += delta
                any_accepted[i] = True
            self.accepted += len(decisions)
            if t == stop_after:
                self.mid = (O.copy(), self.f.copy(), self.evaluated, self.accepted)
        if self.fi:
            self.forced_improvement(O, eq, any_accepted, order)
        self.P = O
        b = int(np.argmax(self.f))
        if self.f[b] > self.fE:
            self.E, self.fE = self.P[b].copy(), int(self.f[b])
        self.gen += 1

    def forced_improvement(self, O, eq, any_accepted, order):
        """Forced improvement as Section 4 describes the serial procedure: a solution with no
        accepted variation in this generation takes the elitist's genes set after set (here in
        the generation's class order, sets of a class ascending), each kept under the usual
        acceptance rule; the first change that raises its fitness ends the procedure, and if
        none does the solution becomes a copy of the elitist."""
        for i in range(self.N):
            if any_accepted[i]:
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
                    delta = self.objective(trial) - self.objective(O[i])
                    if self.may_accept(delta, eq[i]):
                        O[i] = trial
                        self.f[i] += delta
                        self.accepted += 1
                    if delta > 0 or (self.fi_stop_on_accept and self.may_accept(delta, eq[i])):
                        done = True
                        break
                if done:
                    break
            if not done:
                O[i] = self.E
                self.f[i] = self.fE
