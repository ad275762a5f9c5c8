"""CMA-ES reference-parameter search (the paper's Sec. II C: before relative binning can be
used on real data, a covariance-matrix-adaptation evolution strategy maximises the full-band
likelihood to give theta_ref).  TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The strategy is Hansen's (mu/mu_w, lambda)-CMA-ES with cumulative step-size adaptation, in
the notation of N. Hansen, "The CMA Evolution Strategy: A Tutorial" (2016), written here for
maximisation:
  sample     y_k = A z_k,  x_k = m + sigma y_k,  z_k ~ N(0, I) (given),  A A^T = C (Cholesky),
  select     the mu best of the lambda candidates, weights w_i ∝ ln(mu + 1/2) - ln i (sum 1),
  mean       <y>_w = sum_i w_i y_{i:lambda},  m <- m + sigma <y>_w,
  step path  p_s <- (1 - c_s) p_s + sqrt(c_s (2 - c_s) mu_eff) A^{-1} <y>_w,
  step size  sigma <- sigma exp((c_s / d_s) (|p_s| / E|N(0, I)| - 1)),
  cov. path  p_c <- (1 - c_c) p_c + h_s sqrt(c_c (2 - c_c) mu_eff) <y>_w,
  covariance C <- (1 - c_1 - c_mu) C + c_1 (p_c p_c^T + (1 - h_s) c_c (2 - c_c) C)
                  + c_mu sum_i w_i y_{i:lambda} y_{i:lambda}^T,
with the tutorial's default constants.  The search stops (the tutorial's ConditionCov and
TolUpSigma criteria, on the Cholesky factor) once C can no longer be factored, (max_i A_ii /
min_i A_ii)^2 exceeds 1e14, or the largest step sigma max_i A_ii exceeds the box width.  One reading: the tutorial's C^{-1/2} in the step-size
path is taken as A^{-1}, the inverse of the lower Cholesky factor, so that sampling needs no
eigendecomposition (A^{-1} y_k = z_k has the same N(0, I) law under random selection).  The
search runs in box-normalised coordinates u = (theta - lo) / (hi - lo); a candidate outside
the box ranks below every candidate inside it.  Ties keep the candidates' order.

The search is a multistart: independent runs from given starting points, the best candidate
over all of them kept (a long inspiral's likelihood has many separated local maxima along the
chirp-mass / coalescence-time ridge and over the sky; one run ends in whichever it meets
first).
"""
import numpy as np


class CMAES:
    def __init__(self, mean0, sigma0, lam):
        n = len(mean0)
        self.n, self.lam = n, lam
        self.mu = lam // 2
        w = np.log(self.mu + 0.5) - np.log(np.arange(1, self.mu + 1))
        self.w = w / w.sum()
        self.mueff = 1.0 / np.sum(self.w ** 2)
        self.cc = (4.0 + self.mueff / n) / (n + 4.0 + 2.0 * self.mueff / n)
        self.cs = (self.mueff + 2.0) / (n + self.mueff + 5.0)
        self.c1 = 2.0 / ((n + 1.3) ** 2 + self.mueff)
        self.cmu = min(1.0 - self.c1, 2.0 * (self.mueff - 2.0 + 1.0 / self.mueff) / ((n + 2.0) ** 2 + self.mueff))
        self.ds = 1.0 + 2.0 * max(0.0, np.sqrt((self.mueff - 1.0) / (n + 1.0)) - 1.0) + self.cs
        self.chi_n = np.sqrt(n) * (1.0 - 1.0 / (4.0 * n) + 1.0 / (21.0 * n * n))
        self.m = np.array(mean0, dtype=np.float64)
        self.sigma = float(sigma0)
        self.C = np.eye(n)
        self.ps = np.zeros(n)
        self.pc = np.zeros(n)
        self.gen = 0
        self._y = None

    def factor(self):
        """Cholesky factor A of C; False when the search must stop (C not positive definite
        in floating point, or its conditioning beyond 1e14)."""
        try:
            self.A = np.linalg.cholesky(self.C)
        except np.linalg.LinAlgError:
            return False
        d = np.diag(self.A)
        return bool((d.max() / d.min()) ** 2 <= 1e14 and self.sigma * d.max() <= 1.0)

    def ask(self, z):
        """Candidates x_k = m + sigma A z_k for the given standard normals z [lambda, n]."""
        self.A = np.linalg.cholesky(self.C)
        self._y = z @ self.A.T
        return self.m + self.sigma * self._y

    def tell(self, fitness):
        """Update from the candidates' fitness [lambda] (larger is better)."""
        order = np.argsort(-np.asarray(fitness, dtype=np.float64), kind="stable")[: self.mu]
        ysel = self._y[order]
        yw = self.w @ ysel
        self.m = self.m + self.sigma * yw
        zw = np.linalg.solve(self.A, yw)
        n = self.n
        self.ps = (1.0 - self.cs) * self.ps + np.sqrt(self.cs * (2.0 - self.cs) * self.mueff) * zw
        self.gen += 1
        norm_ps = np.linalg.norm(self.ps)
        hs = norm_ps / np.sqrt(1.0 - (1.0 - self.cs) ** (2 * self.gen)) < (1.4 + 2.0 / (n + 1.0)) * self.chi_n
        self.pc = (1.0 - self.cc) * self.pc + (np.sqrt(self.cc * (2.0 - self.cc) * self.mueff) * yw if hs else 0.0)
        rank_mu = (ysel.T * self.w) @ ysel
        self.C = ((1.0 - self.c1 - self.cmu) * self.C
                  + self.c1 * (np.outer(self.pc, self.pc) + (0.0 if hs else self.cc * (2.0 - self.cc)) * self.C)
                  + self.cmu * rank_mu)
        self.C = 0.5 * (self.C + self.C.T)
        self.sigma *= np.exp((self.cs / self.ds) * (norm_ps / self.chi_n - 1.0))


def search(fitness_fn, lo, hi, starts, sigma0, lam, normals):
    """Maximise fitness_fn(theta [k, 13]) -> [k] over the box [lo, hi] by independent runs,
    run r from starts[r] ([n_starts, 13]) with the standard normals normals[r]
    ([n_starts, generations, lambda, 13]).  The runs advance together (one fitness call per
    generation for the candidates of every run still going); run r ends early when its
    covariance's conditioning stops it (CMAES.factor).  Returns (best theta over all runs, its
    fitness, traces: one array [generations run, 2 + 13] per run of (the run's best fitness so
    far, sigma, mean theta)).  On a tie the first candidate seen is kept, runs in order."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    starts = np.atleast_2d(np.asarray(starts, float))
    width = hi - lo
    runs = [CMAES((st - lo) / width, sigma0, lam) for st in starts]
    going = [True] * len(runs)
    run_best = [-np.inf] * len(runs)
    best_f, best_x = -np.inf, starts[0].copy()
    traces = [[] for _ in runs]
    for g in range(normals.shape[1]):
        for r, es in enumerate(runs):
            if going[r] and not es.factor():
                going[r] = False
        active = [r for r in range(len(runs)) if going[r]]
        if not active:
            break
        u = np.concatenate([runs[r].ask(normals[r, g]) for r in active])
        inside = np.all((u >= 0.0) & (u <= 1.0), axis=1)
        theta = lo + u * width
        f = np.full(len(u), -np.inf)
        if inside.any():
            f[inside] = fitness_fn(theta[inside])
        f = np.where(np.isnan(f), -np.inf, f)
        for j, r in enumerate(active):
            fr = f[j * lam:(j + 1) * lam]
            k = int(np.argmax(fr))
            run_best[r] = max(run_best[r], fr[k])
            if fr[k] > best_f:
                best_f, best_x = float(fr[k]), theta[j * lam + k].copy()
            runs[r].tell(fr)
            traces[r].append(np.concatenate([[run_best[r], runs[r].sigma], lo + runs[r].m * width]))
    return best_x, best_f, [np.array(t).reshape(-1, 2 + len(lo)) for t in traces]
