"""The per-frame online PARAFAC step in FP64 (oracle; test infrastructure only).

Single-coil tomographic form: Algorithm 3 with C = 1 and the all-ones coil map,
so the sketch of pixel-domain factors a_r (N1) and b_r (N2) at k-space entry
(i, j) is [F(a_r b_r^T)]_{ij} with F(X) = F_l X F_r (Sec. IV).  One ``push`` is
one pass of the for-loop of Algorithm 3 at time t:

  S1  Phi_t from the factors at t-1, gamma_t = (Phi^H Phi + lambda I)^{-1} Phi^H y
      (closed form of the ridge problem, Sec. III-A), residual e = y - Phi gamma.
  S2  Theta = F^{-1}(Xi) with Xi the zero-filled residual (Sec. IV-B), then
      a_r <- (1 - lambda mu_t / t) a_r + mu_t conj(gamma_r) Theta conj(b_r)
      b_r <- (1 - lambda mu_t / t) b_r + mu_t conj(gamma_r) Theta^T conj(a_r)
      both from the factors at t-1 (Algorithm 3, S2).
  out X_t = A[t] diag(gamma_t) B[t]^T (Sec. IV-A's interpolated frame).

Step size (Sec. III-A, eq. 6): mu_t = 1 / alpha_bar_t, alpha_bar_t = sum of
alpha_tau, with alpha_t at least the largest Hessian eigenvalue of f_t in each
factor.  Reading: alpha_t = lambda/t + max(Gersh(G^H B^H B G), Gersh(G^H A^H A G))
with G = diag(gamma_t) and Gersh(M) = max_r sum_s |M_rs|; since the sampling
projection and F are non-expansive this bounds the factor-block Lipschitz
constant for every mask.  A constant step (the experiments' mu = 0.01, Sec. VI-A)
is the alternative mode.

Other readings: complex data, so every transpose that meets data in S1 is a
Hermitian transpose (Phi^H) while the B^T of the synthesis and the Theta^T of the
B update stay plain transposes; lambda in the ridge (the text's lambda_* is
undefined); t counts every pushed frame from 1; the B update uses the old A
(both updates read the factors at t-1); an empty sample set gives gamma = 0
and a pure shrink; a singular Gram with lambda = 0 is an error, not a choice
among minimisers.
"""

import numpy as np

from .dft import dft_matrix


class NotPositiveDefinite(ValueError):
    """The ridge Gram Phi^H Phi + lambda I is not positive definite."""


class NonFinite(ValueError):
    """A sample or a result is NaN or infinite."""


def regression_matrix(A, B, oi, oj, Fl, Fr):
    """[Phi]_{l, r} = [F(a_r b_r^T)]_{i_l, j_l} for the sampled entries (Alg. 3, S1).

    F(a b^T) = F_l (a b^T) F_r = (F_l a)(b^T F_r) by associativity of the
    matrix products, so column r of Phi is the outer product of F_l a_r and
    b_r^T F_r read at the sampled (i, j).
    """
    FlA = Fl @ A            # column r: F_l a_r
    BtFr = B.T @ Fr         # row r:    b_r^T F_r
    return FlA[oi, :] * BtFr[:, oj].T


def ridge_gamma(Phi, y, lam):
    """Closed form of the S1 ridge problem (Sec. III-A) via a Cholesky solve.

    Returns (gamma, G, h) with G = Phi^H Phi + lambda I and h = Phi^H y.
    Raises NotPositiveDefinite when G has no Cholesky factor.
    """
    R = Phi.shape[1]
    G = Phi.conj().T @ Phi + lam * np.eye(R)
    h = Phi.conj().T @ y
    try:
        L = np.linalg.cholesky(G)
    except np.linalg.LinAlgError as exc:
        raise NotPositiveDefinite(str(exc)) from None
    z = np.linalg.solve(L, h)                 # L z = h
    gamma = np.linalg.solve(L.conj().T, z)    # L^H gamma = z
    return gamma, G, h


def ridge_gamma_svd(Phi, y, lam):
    """The SVD form of the same ridge solution (Algorithm 3, S1).

    With Phi = U Sigma V^H, gamma = V diag(sigma / (sigma^2 + lambda)) U^H y.
    """
    U, s, Vh = np.linalg.svd(Phi, full_matrices=False)
    return Vh.conj().T @ ((s / (s * s + lam)) * (U.conj().T @ y))


def gram_pivot_ratio(G):
    """max_k D_k / min_k D_k over the pivots of G = L D L^H (D_k = |L_kk|^2 of the
    Cholesky factor): the conditioning figure reported per frame for the ridge
    Gram of Sec. III-A.  Every pivot is a Schur complement's diagonal entry and
    lies in [lambda_min(G), lambda_max(G)], so the ratio never exceeds
    kappa_2(G), and equals it when G is diagonal."""
    L = np.linalg.cholesky(G)
    d = np.abs(np.diag(L)) ** 2
    return float(d.max() / d.min())


def back_projection(Xi, Fl, Fr):
    """Theta = F^{-1}(Xi) = F_l^H Xi F_r^H (Sec. IV-B with one coil, H = ones)."""
    return Fl.conj().T @ Xi @ Fr.conj().T


def gershgorin(M):
    """max_r sum_s |M_rs|, an upper bound on the spectral radius of M."""
    return float(np.max(np.sum(np.abs(M), axis=1))) if M.size else 0.0


def step_alpha(A, B, gamma, lam, t):
    """alpha_t of the majorizer (Sec. III-A): lambda/t + largest factor-block bound."""
    Gc = np.diag(gamma)
    MB = Gc.conj().T @ (B.conj().T @ B) @ Gc
    MA = Gc.conj().T @ (A.conj().T @ A) @ Gc
    return lam / t + max(gershgorin(MB), gershgorin(MA))


def instantaneous_cost(A, B, gamma, oi, oj, y, lam, t, Fl, Fr):
    """f_t(A, B; gamma) of eq. (5): half the squared fit plus (lambda/2t) sum ||A_m||^2."""
    Phi = regression_matrix(A, B, oi, oj, Fl, Fr)
    r = y - Phi @ gamma
    return 0.5 * float(np.vdot(r, r).real) + (lam / (2.0 * t)) * (
        float(np.vdot(A, A).real) + float(np.vdot(B, B).real))


class Step:
    """Everything one push produced (attributes named as in the paper)."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def _omega_lines(rows, n2):
    rows = np.asarray(rows, dtype=np.int64)
    oi = np.repeat(rows, n2)
    oj = np.tile(np.arange(n2, dtype=np.int64), rows.size)
    return oi, oj


def _check_lines(rows, n1):
    rows = np.asarray(rows, dtype=np.int64)
    if rows.ndim != 1 or np.any(rows < 0) or np.any(rows >= n1) or np.any(np.diff(rows) <= 0):
        raise ValueError("rows must be ascending, unique and inside [0, n1)")
    return rows


class TslOracle:
    """State (A, B, alpha_bar, t) and the per-frame step of Algorithm 3, C = 1."""

    def __init__(self, n1, n2, r, lam, A0, B0, step_mode="mm", mu=None):
        self.n1, self.n2, self.r, self.lam = int(n1), int(n2), int(r), float(lam)
        self.A = np.array(A0, dtype=np.complex128).reshape(n1, r)
        self.B = np.array(B0, dtype=np.complex128).reshape(n2, r)
        if step_mode not in ("mm", "const"):
            raise ValueError("step_mode is 'mm' or 'const'")
        if step_mode == "const" and (mu is None or not mu > 0):
            raise ValueError("constant step needs mu > 0")
        self.step_mode, self.mu_const = step_mode, mu
        self.abar = 0.0
        self.t = 0
        self.Fl = dft_matrix(self.n1)
        self.Fr = dft_matrix(self.n2)

    # --- the factor transforms the sampler and the k-space view use -------------
    def kspace_factors(self):
        """(F_l A, F_r B): the k-space row factors (Sec. IV-A, Algorithm 2's factors)."""
        return self.Fl @ self.A, self.Fr @ self.B

    # --- one frame -------------------------------------------------------------
    def push_lines(self, rows, Y):
        """Frame whose sample set is the full rows ``rows`` (ascending, unique);
        ``Y`` is [len(rows), n2] with Y[s] the samples of row rows[s]."""
        rows = _check_lines(rows, self.n1)
        Y = np.asarray(Y).reshape(rows.size, self.n2)
        oi, oj = _omega_lines(rows, self.n2)
        return self._push(oi, oj, Y.reshape(-1).astype(np.complex128))

    def push_points(self, mask, Y):
        """Frame whose sample set is the boolean [n1, n2] ``mask``; ``Y`` is a full
        [n1, n2] array of which only the masked entries are read."""
        mask = np.asarray(mask, dtype=bool).reshape(self.n1, self.n2)
        oi, oj = np.nonzero(mask)
        return self._push(oi, oj, np.asarray(Y).reshape(self.n1, self.n2)[oi, oj].astype(np.complex128))

    def _push(self, oi, oj, y):
        if not np.all(np.isfinite(y)):
            raise NonFinite("non-finite sample")
        t = self.t + 1
        A, B, lam = self.A, self.B, self.lam

        # S1: principal components from the factors at t-1.
        Phi = regression_matrix(A, B, oi, oj, self.Fl, self.Fr)
        gamma, G, h = ridge_gamma(Phi, y, lam)
        e = y - Phi @ gamma
        Xi = np.zeros((self.n1, self.n2), dtype=np.complex128)
        Xi[oi, oj] = e

        # Step size of the majorization-minimization recursion.
        alpha = step_alpha(A, B, gamma, lam, t)
        abar = self.abar + alpha
        mu = 1.0 / abar if self.step_mode == "mm" else float(self.mu_const)

        # S2: parallel subspace update from the factors at t-1.
        Theta = back_projection(Xi, self.Fl, self.Fr)
        shrink = 1.0 - lam * mu / t
        cg = np.conj(gamma)[None, :]
        A_new = shrink * A + mu * (Theta @ np.conj(B)) * cg
        B_new = shrink * B + mu * (Theta.T @ np.conj(A)) * cg
        X = A_new @ np.diag(gamma) @ B_new.T
        if not (np.all(np.isfinite(A_new)) and np.all(np.isfinite(B_new))):
            raise NonFinite("non-finite factor update")

        self.A, self.B, self.abar, self.t = A_new, B_new, abar, t
        return Step(t=t, gamma=gamma, G=G, h=h, e=e, Xi=Xi, Theta=Theta, alpha=alpha,
                    alpha_bar=abar, mu=mu, shrink=shrink, A=A_new, B=B_new, X=X,
                    oi=oi, oj=oj, y=y, pivot_ratio=gram_pivot_ratio(G))


class KspaceOracle:
    """Algorithm 2 (online k-space interpolation) on k-space factors (alpha, beta).

    The sketch of entry (i, j) is alpha_{ir} beta_{jr} with W = e_i e_j^T, the
    ridge and step-size rules are those of TslOracle, and the row-wise updates are
      alpha_r <- (1 - lambda mu/t) alpha_r + mu conj(gamma_r) sum_{(i,j)} e_ij conj(beta_jr) e_i
      beta_r  <- (1 - lambda mu/t) beta_r  + mu conj(gamma_r) sum_{(i,j)} e_ij conj(alpha_ir) e_j.
    It shares only the ridge and step-size helpers with TslOracle; started from
    (F_l A0, F_r B0) it is an independent formulation of the same iterates.
    """

    def __init__(self, n1, n2, r, lam, alpha0, beta0, step_mode="mm", mu=None):
        self.n1, self.n2, self.r, self.lam = int(n1), int(n2), int(r), float(lam)
        self.alpha = np.array(alpha0, dtype=np.complex128).reshape(n1, r)
        self.beta = np.array(beta0, dtype=np.complex128).reshape(n2, r)
        self.step_mode, self.mu_const = step_mode, mu
        self.abar = 0.0
        self.t = 0

    def push_lines(self, rows, Y):
        rows = _check_lines(rows, self.n1)
        oi, oj = _omega_lines(rows, self.n2)
        return self._push(oi, oj, np.asarray(Y).reshape(-1).astype(np.complex128))

    def push_points(self, mask, Y):
        oi, oj = np.nonzero(np.asarray(mask, dtype=bool).reshape(self.n1, self.n2))
        return self._push(oi, oj, np.asarray(Y).reshape(self.n1, self.n2)[oi, oj].astype(np.complex128))

    def _push(self, oi, oj, y):
        t = self.t + 1
        al, be, lam = self.alpha, self.beta, self.lam
        Phi = al[oi, :] * be[oj, :]
        gamma, G, h = ridge_gamma(Phi, y, lam)
        e = y - Phi @ gamma
        alpha = step_alpha(al, be, gamma, lam, t)
        abar = self.abar + alpha
        mu = 1.0 / abar if self.step_mode == "mm" else float(self.mu_const)
        shrink = 1.0 - lam * mu / t
        cg = np.conj(gamma)[None, :]
        ga = np.zeros_like(al)
        gb = np.zeros_like(be)
        np.add.at(ga, oi, e[:, None] * np.conj(be[oj, :]))
        np.add.at(gb, oj, e[:, None] * np.conj(al[oi, :]))
        al_new = shrink * al + mu * ga * cg
        be_new = shrink * be + mu * gb * cg
        self.alpha, self.beta, self.abar, self.t = al_new, be_new, abar, t
        Xk = al_new @ np.diag(gamma) @ be_new.T
        return Step(t=t, gamma=gamma, alpha_f=al_new, beta_f=be_new, Xk=Xk,
                    alpha=alpha, alpha_bar=abar, mu=mu)


def epochs(ora, frames, order):
    """Batch processing of a stored scan in several passes (Sec. VI-D).

    ``frames[k]`` is ("lines", rows, Y) or ("points", mask, Y); pass e visits
    the frames in the order ``order[e]`` (a permutation of range(T)), each visit
    one push of ``ora`` with its state carried over from the previous visit (the
    subspace learnt in a pass starts the next one).  Returns the step of each
    frame's last visit."""
    T = len(frames)
    last = [None] * T
    for perm in order:
        perm = [int(v) for v in perm]
        if sorted(perm) != list(range(T)):
            raise ValueError("each pass must be a permutation of range(T)")
        for v in perm:
            kind, sel, Y = frames[v]
            last[v] = ora.push_lines(sel, Y) if kind == "lines" else ora.push_points(sel, Y)
    return last


# ---------------------------------------------------------------- several coils (Sec. IV-B)
def coil_regression_matrix(A, B, H, rows, Fl, Fr):
    """[Phi]_{(c, i, j), r} = [F(H_c .* (a_r b_r^T))]_{ij} for the sampled rows
    (every column of each), coils stacked in order (Algorithm 3, S1).  H is
    [C, N1, N2]; returns [C * len(rows) * N2, R]."""
    C = H.shape[0]
    R = A.shape[1]
    out = []
    for c in range(C):
        cols = [(Fl @ (H[c] * np.outer(A[:, r], B[:, r])) @ Fr)[rows, :].reshape(-1) for r in range(R)]
        out.append(np.stack(cols, axis=1))
    return np.concatenate(out, axis=0)


def coil_gain(H):
    """max over pixels of sum_c |H_c|^2: the factor by which the coil-weighted
    sampling can stretch a frame's norm (1 for a single all-ones map)."""
    return float(np.max(np.sum(np.abs(H) ** 2, axis=0)))


class CoilOracle:
    """Algorithm 3 with C coils and sensitivity maps H_c (Sec. IV-B), line masks.

    Per frame: Phi from F(H_c .* (a_r b_r^T)) at the sampled rows of every coil,
    gamma the ridge solution over all coils' samples, the residual e_c per coil,
    Theta = sum_c conj(H_c) .* F^{-1}(Xi_c) (Xi_c the zero-filled residual of
    coil c) and the S2 updates of Algorithm 3 from the factors at t-1.  Step
    size (reading): alpha_t = lambda/t + g max(Gersh(G^H B^H B G), Gersh(G^H A^H A G))
    with g = max over pixels of sum_c |H_c|^2, which bounds the factor-block
    Lipschitz constant since ||P F(H_c .* X)|| <= ||H_c .* X|| and
    sum_c ||H_c .* X||^2 <= g ||X||^2; with one all-ones map it is the
    single-coil rule.  Output X_t = A[t] diag(gamma_t) B[t]^T."""

    def __init__(self, n1, n2, r, lam, A0, B0, H, step_mode="mm", mu=None):
        self.n1, self.n2, self.r, self.lam = int(n1), int(n2), int(r), float(lam)
        self.A = np.array(A0, dtype=np.complex128).reshape(n1, r)
        self.B = np.array(B0, dtype=np.complex128).reshape(n2, r)
        self.H = np.array(H, dtype=np.complex128).reshape(-1, n1, n2)
        self.C = self.H.shape[0]
        self.step_mode, self.mu_const = step_mode, mu
        self.abar, self.t = 0.0, 0
        self.Fl, self.Fr = dft_matrix(self.n1), dft_matrix(self.n2)
        self.gain = coil_gain(self.H)

    def kspace_factors(self):
        return self.Fl @ self.A, self.Fr @ self.B

    def push_lines(self, rows, Y):
        """``Y`` is [C, len(rows), n2]: Y[c, s] the samples of row rows[s] at coil c."""
        rows = _check_lines(rows, self.n1)
        Y = np.asarray(Y).reshape(self.C, rows.size, self.n2).astype(np.complex128)
        if not np.all(np.isfinite(Y)):
            raise NonFinite("non-finite sample")
        t = self.t + 1
        A, B, lam = self.A, self.B, self.lam
        Phi = coil_regression_matrix(A, B, self.H, rows, self.Fl, self.Fr)
        y = Y.reshape(-1)
        gamma, G, h = ridge_gamma(Phi, y, lam)
        e = (y - Phi @ gamma).reshape(self.C, rows.size, self.n2)
        Theta = np.zeros((self.n1, self.n2), dtype=np.complex128)
        for c in range(self.C):
            Xi = np.zeros((self.n1, self.n2), dtype=np.complex128)
            Xi[rows, :] = e[c]
            Theta += np.conj(self.H[c]) * back_projection(Xi, self.Fl, self.Fr)
        alpha = lam / t + self.gain * (step_alpha(A, B, gamma, 0.0, t))
        abar = self.abar + alpha
        mu = 1.0 / abar if self.step_mode == "mm" else float(self.mu_const)
        shrink = 1.0 - lam * mu / t
        cg = np.conj(gamma)[None, :]
        A_new = shrink * A + mu * (Theta @ np.conj(B)) * cg
        B_new = shrink * B + mu * (Theta.T @ np.conj(A)) * cg
        X = A_new @ np.diag(gamma) @ B_new.T
        self.A, self.B, self.abar, self.t = A_new, B_new, abar, t
        return Step(t=t, gamma=gamma, G=G, h=h, e=e, Theta=Theta, alpha=alpha, alpha_bar=abar, mu=mu,
                    shrink=shrink, A=A_new, B=B_new, X=X, Phi=Phi, y=y)
