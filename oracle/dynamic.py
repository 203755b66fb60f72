"""Static CSC and dynamic CSC (Algorithm 1 of Sec. 4.1), in FP64.

Static CSC (Sec. 2.2, Step 1 with lambda_k from an eigencount dichotomy): filter d
Gaussian signals of variance 1/d with the polynomial low-pass at lambda_k and run
k-means on the rows.

Dynamic CSC keeps, at snapshot t >= 2, a fraction p of the filtered columns of earlier
snapshots and filters only q d = (1 - p) d fresh signals on G_t with the previous
filter h^{t-1} (eq. features_f).  The eigencount of those fresh columns decides whether
h^{t-1} still fits G_t; if not, lambda is refined by a dichotomy that starts from the
previous value and the fresh columns are filtered again.  k-means then runs on the
combined features.

Readings where the paper is silent or leaves a choice
  * snapshot 1 uses the d feature columns themselves as eigencount probes;
  * the d columns form a FIFO ring at column granularity: the q d columns filtered longest
    ago are replaced, starting at a cursor that advances by q d modulo d (a block may wrap
    around the last column); for p <= 1/2 the kept columns always come from G_{t-1}, as
    the paper assumes, and for p > 1/2 columns live for up to ceil(p / q) snapshots;
  * acceptance |c - k| <= tau with tau = max(0.5, 2 sqrt(2 k / (q d)));
  * refinement bisects [lambda_{t-1}, lmax] when c < k and [0, lambda_{t-1}] otherwise;
  * random draws come from Philox4x32-10 with stream id 16 t + purpose (signals 1,
    k-means uniforms 2), see :mod:`oracle.philox`;
  * k-means: k-means++ seeding then a fixed number of Lloyd rounds, or a warm start
    from the previous labels (means of the new features under the old labels);
  * with the combinatorial Laplacian D - W and no lmax given, each snapshot maps its own
    spectrum bound (Anderson-Morley, :mod:`oracle.operator`) onto [-1, 1]; lambda_{t-1}
    is an absolute cut-off, clipped to the new bound where a bracket needs it;
  * similarity (Sec. 4 metrics): each snapshot t >= 2 reports ||L_t - L_{t-1}||_F and, with
    sim_probes = s > 0, the estimate rho_hat of the spectral distance from the first s fresh
    signals filtered with h^{t-1} on both graphs (:mod:`oracle.similarity`); with a
    refresh budget, a snapshot where p * rho_hat exceeds it is processed as static CSC (all d
    columns drawn from its signal stream, the ring restarts).  Thm 4.1 bounds the reuse term
    by (1 + delta) p rho; the rule keeps that term under the budget.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import chebyshev, eigcount, kmeans, operator, philox, similarity

SIGNALS = 1
KMEANS = 2


def stream_id(t: int, purpose: int) -> int:
    return 16 * int(t) + int(purpose)


@dataclass
class StepResult:
    t: int
    lam: float
    count: float
    refined: bool
    labels: np.ndarray
    centroids: np.ndarray
    objective: list = field(default_factory=list)
    rho_edge: float = -1.0      # ||L_t - L_{t-1}||_F (t >= 2)
    rho_hat: float = -1.0       # filtered-signal estimate of the spectral distance, if asked
    refreshed: bool = False     # all d columns recomputed by the refresh rule


def run_kmeans(F: np.ndarray, k: int, iters: int, seed: int, t: int, init: str,
               prev_labels: np.ndarray | None):
    if init == "warm" and prev_labels is not None:
        C0, _ = kmeans.update(F, prev_labels, np.zeros((k, F.shape[1])))
    else:
        u = philox.uniforms(k, seed, stream_id(t, KMEANS))
        C0 = np.asarray(F, dtype=np.float64)[kmeans.kmeanspp(F, k, u)]
    return kmeans.lloyd(F, C0, iters)


class DynamicCSC:
    def __init__(self, n: int, d: int, k: int, p: float, m: int, seed: int,
                 lmax: float | None = None, damping: str = "jackson", n_cand: int = 16,
                 lloyd_iters: int = 20, tau: float | None = None, init: str = "kmeans++",
                 storage=np.float64, laplacian: str = "normalized",
                 sim_probes: int = 0, refresh_budget: float | None = None):
        self.n, self.d, self.k, self.p, self.m = n, d, k, p, m
        self.qd = int(round((1.0 - p) * d))
        if self.qd < 1 or self.qd > d:
            raise ValueError("need 1 <= (1 - p) d <= d")
        if laplacian not in ("normalized", "combinatorial"):
            raise ValueError(laplacian)
        self.laplacian = laplacian
        if not 0 <= sim_probes <= self.qd:
            raise ValueError("need 0 <= sim_probes <= (1 - p) d")
        self.sim_probes = sim_probes
        self.refresh_budget = refresh_budget
        self.prev = None            # (operator, lmax) of G_{t-1}
        self.seed = seed
        self.lmax = lmax
        self.damping = damping
        self.n_cand = n_cand
        self.lloyd_iters = lloyd_iters
        self.tau = eigcount.accept_tolerance(k, self.qd) if tau is None else tau
        self.init = init
        self.storage = storage
        self.sigma = 1.0 / np.sqrt(d)
        self.theta = np.zeros((n, d))
        self.t = 0
        self.lam = None
        self.cursor = 0
        self.labels = None

    def _signals(self, w: int, t: int) -> np.ndarray:
        R = philox.gaussian_block(self.n, w, self.sigma, self.seed, stream_id(t, SIGNALS),
                                  dtype=self.storage)
        return np.asarray(R, dtype=np.float64)

    def step(self, g) -> StepResult:
        """Process the next snapshot, given as a CSR weight matrix (workloads.Graph)."""
        if self.laplacian == "normalized":
            A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
            lmax = self.lmax if self.lmax is not None else 2.0
        else:
            A = operator.combinatorial_laplacian(g.n, g.rowptr, g.colidx, g.w)
            lmax = self.lmax if self.lmax is not None else \
                operator.anderson_morley_bound(g.n, g.rowptr, g.colidx, g.w)
        self.t += 1
        t = self.t
        sigma2 = self.sigma ** 2
        rho_edge = rho_hat = -1.0
        refreshed = False
        if t == 1:
            lam, cnt = self._static(A, lmax, t)
            refined = True
        else:
            R = self._signals(self.qd, t)
            a = chebyshev.step_coefficients(self.m, lmax, self.lam, self.damping)
            Y = chebyshev.filter_recurrence(A, lmax, a, R)
            cnt = float(np.sum(R * Y) / (sigma2 * self.qd))
            lam = self.lam
            refined = False
            # similarity of G_t to G_{t-1} (Sec. 4 metrics), and the refresh rule of Thm 4.1:
            # the reuse term grows like p * rho, so a snapshot whose estimated spectral
            # distance exceeds budget / p recomputes every feature
            A_prev, lmax_prev = self.prev
            rho_edge = similarity.edge_distance(A_prev, A)
            if self.sim_probes > 0:
                s_ = self.sim_probes
                a_prev = chebyshev.step_coefficients(self.m, lmax_prev, min(self.lam, lmax_prev),
                                                     self.damping)
                Y_prev = chebyshev.filter_recurrence(A_prev, lmax_prev, a_prev, R[:, :s_])
                rho_hat = float(np.sqrt(np.sum((Y[:, :s_] - Y_prev) ** 2) / (sigma2 * s_)))
            if (self.refresh_budget is not None and rho_hat >= 0.0
                    and self.p * rho_hat > self.refresh_budget):
                lam, cnt = self._static(A, lmax, t)
                refined = refreshed = True
            else:
                if abs(cnt - self.k) > self.tau:
                    mu = eigcount.moments_direct(A, lmax, self.m, R)
                    prev = min(self.lam, lmax)
                    lo, hi = (prev, lmax) if cnt < self.k else (0.0, prev)
                    lam, cnt, _ = eigcount.eigcount_bisect(mu, self.m, lmax, self.damping,
                                                           sigma2, self.qd, self.k, self.n_cand,
                                                           lo, hi)
                    a = chebyshev.step_coefficients(self.m, lmax, lam, self.damping)
                    Y = chebyshev.filter_recurrence(A, lmax, a, R)
                    refined = True
                cols = (self.cursor + np.arange(self.qd)) % self.d
                self.theta[:, cols] = Y
                self.cursor = (self.cursor + self.qd) % self.d
        self.lam = lam
        self.prev = (A, lmax)
        lab, C, obj = run_kmeans(self.theta, self.k, self.lloyd_iters, self.seed, t,
                                 self.init, self.labels)
        self.labels = lab
        return StepResult(t=t, lam=lam, count=cnt, refined=refined, labels=lab,
                          centroids=C, objective=obj, rho_edge=rho_edge, rho_hat=rho_hat,
                          refreshed=refreshed)

    def _static(self, A, lmax: float, t: int):
        """Static CSC on this snapshot: d signals, their moments as eigencount probes, the
        dichotomy on [0, lmax], the filter at the found cut-off; the ring restarts."""
        sigma2 = self.sigma ** 2
        R = self._signals(self.d, t)
        mu = eigcount.moments_direct(A, lmax, self.m, R)
        lam, cnt, _ = eigcount.eigcount_bisect(mu, self.m, lmax, self.damping, sigma2, self.d,
                                               self.k, self.n_cand, 0.0, lmax)
        a = chebyshev.step_coefficients(self.m, lmax, lam, self.damping)
        self.theta = chebyshev.filter_recurrence(A, lmax, a, R)
        self.cursor = 0
        return lam, cnt
