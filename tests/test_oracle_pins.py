"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these checks retypes the oracle's own formula: each compares it with an
independent route (a library transform, an explicit sketch-matrix sum, a finite
difference, a brute-force eigenvalue, a closed form, a published known-answer
table, a second formulation of the algorithm, or a statistical law).
"""

import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import tsl as otsl
from oracle.sampler import expected_count, point_scores
from paper_1609_04104_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(s):
    return np.random.default_rng(1000 + s)


def _cn(rng, shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def _nr(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


# ----------------------------------------------------------------- DFT (Sec. IV)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 12, 15, 64, 120, 200, 256])
def test_dft_matches_library_fft_unitary_symmetric(n):
    F = oracle.dft_matrix(n)
    x = _cn(_rng(n), n)
    assert np.allclose(F @ x, np.fft.fft(x, norm="ortho"), atol=1e-12, rtol=0)
    assert np.allclose(F, F.T, atol=0, rtol=0)                                    # symmetric
    assert np.allclose(F.conj().T @ F, np.eye(n), atol=1e-12)                     # unitary
    assert abs(np.linalg.norm(F @ x) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)  # Parseval


def test_dft_closed_forms():
    n = 12
    F = oracle.dft_matrix(n)
    d = np.zeros(n); d[0] = 1.0
    assert np.allclose(F @ d, np.full(n, 1.0 / np.sqrt(n)), atol=1e-15)           # delta -> flat
    m0 = 5
    tone = np.exp(2j * np.pi * m0 * np.arange(n) / n)
    expect = np.zeros(n, complex); expect[m0] = np.sqrt(n)
    assert np.allclose(F @ tone, expect, atol=1e-12)                               # tone -> spike


def test_fft2_matches_library_and_inverts():
    rng = _rng(1)
    X = _cn(rng, (24, 40))
    K = oracle.fft2_unitary(X)
    assert np.allclose(K, np.fft.fft2(X, norm="ortho"), atol=1e-12)
    assert np.allclose(oracle.ifft2_unitary(K), X, atol=1e-12)
    a, b = _cn(rng, 24), _cn(rng, 40)
    # separability F(a b^T) = (F_l a)(F_r b)^T, which needs F_r symmetric
    assert np.allclose(oracle.fft2_unitary(np.outer(a, b)),
                       np.outer(oracle.dft_matrix(24) @ a, oracle.dft_matrix(40) @ b), atol=1e-12)


# ----------------------------------------------------------------- S1 (Sec. III-A)
def test_regression_matrix_columns_are_sampled_fft_of_rank_one():
    rng = _rng(2)
    n1, n2, R = 10, 9, 4
    A, B = _cn(rng, (n1, R)), _cn(rng, (n2, R))
    mask = rng.random((n1, n2)) < 0.4
    oi, oj = np.nonzero(mask)
    Phi = oracle.regression_matrix(A, B, oi, oj, oracle.dft_matrix(n1), oracle.dft_matrix(n2))
    for r in range(R):
        col = np.fft.fft2(np.outer(A[:, r], B[:, r]), norm="ortho")[oi, oj]
        assert np.allclose(Phi[:, r], col, atol=1e-12)


def test_ridge_closed_form_equals_svd_form_and_augmented_lstsq():
    rng = _rng(3)
    for L, R, lam in [(50, 8, 0.3), (6, 10, 0.7), (200, 32, 0.05)]:
        Phi, y = _cn(rng, (L, R)), _cn(rng, L)
        g, G, h = oracle.ridge_gamma(Phi, y, lam)
        g_svd = oracle.ridge_gamma_svd(Phi, y, lam)
        aug = np.vstack([Phi, np.sqrt(lam) * np.eye(R)])
        g_ls = scipy.linalg.lstsq(aug, np.concatenate([y, np.zeros(R)]))[0]
        assert _nr(g, g_svd) < 1e-10
        assert _nr(g, g_ls) < 1e-10


def test_ridge_scalar_case_and_limits():
    rng = _rng(4)
    phi, y = _cn(rng, (30, 1)), _cn(rng, 30)
    lam = 0.9
    g, _, _ = oracle.ridge_gamma(phi, y, lam)
    assert np.allclose(g[0], np.vdot(phi[:, 0], y) / (np.vdot(phi[:, 0], phi[:, 0]).real + lam))
    Phi = _cn(rng, (40, 6))
    g_big, _, _ = oracle.ridge_gamma(Phi, _cn(rng, 40), 1e12)
    assert np.linalg.norm(g_big) < 1e-9
    # rank-deficient Phi with lambda = 0 is an error, not an arbitrary choice
    Phi_def = np.hstack([Phi[:, :3], Phi[:, :3]])
    with pytest.raises(otsl.NotPositiveDefinite):
        oracle.ridge_gamma(Phi_def, _cn(rng, 40), 0.0)


# ----------------------------------------------------------------- residual and back-projection
def _tiny_state(seed=5, n1=6, n2=5, R=3):
    rng = _rng(seed)
    return rng, n1, n2, R, 0.2 * _cn(rng, (n1, R)), 0.2 * _cn(rng, (n2, R))


def test_residual_equals_y_minus_fft_of_synthesis():
    rng, n1, n2, R, A, B = _tiny_state()
    o = oracle.TslOracle(n1, n2, R, 0.1, A, B)
    mask = rng.random((n1, n2)) < 0.5
    Y = _cn(rng, (n1, n2))
    s = o.push_points(mask, Y)
    K = np.fft.fft2((A * s.gamma[None, :]) @ B.T, norm="ortho")
    assert np.allclose(s.e, Y[mask] - K[mask], atol=1e-12)


def test_back_projection_equals_explicit_sketch_sum():
    rng, n1, n2, R, A, B = _tiny_state(6)
    Fl, Fr = oracle.dft_matrix(n1), oracle.dft_matrix(n2)
    Xi = np.zeros((n1, n2), complex)
    mask = rng.random((n1, n2)) < 0.5
    Xi[mask] = _cn(rng, mask.sum())
    Theta = np.zeros((n1, n2), complex)
    for i, j in zip(*np.nonzero(mask)):
        E = np.zeros((n1, n2)); E[i, j] = 1.0
        W = Fl @ E @ Fr                          # sketch of entry (i, j)
        Theta += Xi[i, j] * np.conj(W)           # sum_l e_l W_l^*
    assert np.allclose(oracle.back_projection(Xi, Fl, Fr), Theta, atol=1e-12)


# ----------------------------------------------------------------- gradient, Hessian bound, MM
def _explicit_gradient(A, B, gamma, oi, oj, y, lam, t, Fl, Fr, wrt="A"):
    """eq. (7) with explicit sketch matrices W_l = F_l e_i e_j^T F_r."""
    n1, n2 = Fl.shape[0], Fr.shape[0]
    R = A.shape[1]
    Ws = []
    for i, j in zip(oi, oj):
        E = np.zeros((n1, n2)); E[i, j] = 1.0
        Ws.append(Fl @ E @ Fr)
    # <a b^T, W> = sum_mn a_m b_n W_mn (bilinear)
    e = np.array([y[l] - sum(gamma[r] * (A[:, r] @ Ws[l] @ B[:, r]) for r in range(R))
                  for l in range(len(Ws))])
    if wrt == "A":
        g = (lam / t) * A.astype(complex)
        for r in range(R):
            for l, W in enumerate(Ws):
                g[:, r] -= np.conj(gamma[r]) * e[l] * np.conj(W @ B[:, r])
    else:
        g = (lam / t) * B.astype(complex)
        for r in range(R):
            for l, W in enumerate(Ws):
                g[:, r] -= np.conj(gamma[r]) * e[l] * np.conj(W.T @ A[:, r])
    return g


def test_update_direction_is_eq7_gradient_and_matches_finite_differences():
    rng, n1, n2, R, A, B = _tiny_state(7)
    lam = 0.3
    o = oracle.TslOracle(n1, n2, R, lam, A, B)
    o.push_points(rng.random((n1, n2)) < 0.6, _cn(rng, (n1, n2)))   # t = 1, move away from init
    A1, B1 = o.A.copy(), o.B.copy()
    mask = rng.random((n1, n2)) < 0.6
    Y = _cn(rng, (n1, n2))
    s = o.push_points(mask, Y)
    t, Fl, Fr = s.t, o.Fl, o.Fr
    gA = (A1 - s.A) / s.mu
    gB = (B1 - s.B) / s.mu
    assert np.allclose(gA, _explicit_gradient(A1, B1, s.gamma, s.oi, s.oj, s.y, lam, t, Fl, Fr, "A"), atol=1e-10)
    assert np.allclose(gB, _explicit_gradient(A1, B1, s.gamma, s.oi, s.oj, s.y, lam, t, Fl, Fr, "B"), atol=1e-10)
    # directional derivatives by central differences: df = Re <grad, E>
    f = lambda a, b: oracle.instantaneous_cost(a, b, s.gamma, s.oi, s.oj, s.y, lam, t, Fl, Fr)
    for _ in range(3):
        E = _cn(rng, A1.shape)
        h = 1e-6
        fd = (f(A1 + h * E, B1) - f(A1 - h * E, B1)) / (2 * h)
        assert abs(fd - np.vdot(gA, E).real) < 1e-6 * max(1.0, abs(fd))
        E = _cn(rng, B1.shape)
        fd = (f(A1, B1 + h * E) - f(A1, B1 - h * E)) / (2 * h)
        assert abs(fd - np.vdot(gB, E).real) < 1e-6 * max(1.0, abs(fd))


def _block_operator(A, B, gamma, oi, oj, Fl, Fr, wrt):
    """Matrix of the complex-linear map (factor) -> sampled F(A diag(g) B^T)."""
    n = A.shape[0] if wrt == "A" else B.shape[0]
    R = A.shape[1]
    cols = []
    for r in range(R):
        for m in range(n):
            D = np.zeros((n, R), complex); D[m, r] = 1.0
            X = (D * gamma) @ B.T if wrt == "A" else (A * gamma) @ D.T
            cols.append((Fl @ X @ Fr)[oi, oj])
    return np.array(cols).T


@pytest.mark.parametrize("seed", [8, 9, 10])
def test_step_alpha_bounds_the_block_hessian(seed):
    rng, n1, n2, R, A, B = _tiny_state(seed, n1=7, n2=6, R=3)
    Fl, Fr = oracle.dft_matrix(n1), oracle.dft_matrix(n2)
    gamma = _cn(rng, R)
    lam, t = 0.4, 3
    mask = rng.random((n1, n2)) < 0.5
    oi, oj = np.nonzero(mask)
    alpha = oracle.step_alpha(A, B, gamma, lam, t)
    for wrt in ("A", "B"):
        Lop = _block_operator(A, B, gamma, oi, oj, Fl, Fr, wrt)
        H = Lop.conj().T @ Lop + (lam / t) * np.eye(Lop.shape[1])   # Hessian of f_t in this factor
        assert np.linalg.eigvalsh(H).max() <= alpha * (1 + 1e-12)
    # with every entry sampled, the bound is attained up to the Gershgorin slack
    full = np.ones((n1, n2), bool)
    Lop = _block_operator(A, B, gamma, *np.nonzero(full), Fl, Fr, "A")
    top = np.linalg.eigvalsh(Lop.conj().T @ Lop).max() + lam / t
    assert top <= alpha * (1 + 1e-12)


def _orthogonal_columns(rng, n, norms):
    """n x R matrix whose columns are orthogonal with the given Euclidean norms."""
    Q, _ = np.linalg.qr(_cn(rng, (n, len(norms))))
    return Q * np.asarray(norms, float)[None, :]


def _alpha_pin_case(seed, step_alpha):
    """Factors with orthogonal columns, every entry sampled, t = 3.

    There A^H A and B^H B are diagonal, so the Gershgorin bound of eq. (8)'s
    block Hessians is exact and alpha_t must equal the largest eigenvalue of the
    two factor-block Hessians of f_t (eq. 5), found here by brute force from the
    explicit linear map factor -> sampled F(A diag(gamma) B^T).  Returns
    (alpha from `step_alpha`, brute-force top eigenvalue, closed form)."""
    rng = _rng(40 + seed)
    n1, n2, R = 7, 6, 3
    A = _orthogonal_columns(rng, n1, [1.7, 0.6, 1.1])
    B = _orthogonal_columns(rng, n2, [0.5, 1.3, 0.9])
    gamma = _cn(rng, R)
    lam, t = 0.9, 3
    Fl, Fr = oracle.dft_matrix(n1), oracle.dft_matrix(n2)
    oi, oj = np.nonzero(np.ones((n1, n2), bool))
    top = 0.0
    for wrt in ("A", "B"):
        Lop = _block_operator(A, B, gamma, oi, oj, Fl, Fr, wrt)
        H = Lop.conj().T @ Lop + (lam / t) * np.eye(Lop.shape[1])
        top = max(top, float(np.linalg.eigvalsh(H).max()))
    g2 = np.abs(gamma) ** 2
    closed = lam / t + float(np.max(g2 * np.maximum(np.sum(np.abs(A) ** 2, 0), np.sum(np.abs(B) ** 2, 0))))
    return step_alpha(A, B, gamma, lam, t), top, closed


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_step_alpha_equals_block_hessian_top_eigenvalue_when_gershgorin_is_exact(seed):
    alpha, top, closed = _alpha_pin_case(seed, oracle.step_alpha)
    assert abs(top - closed) <= 1e-12 * closed          # the brute force agrees with the closed form
    assert abs(alpha - top) <= 1e-12 * top               # eq. (6)/(8) reading, fixed from above and below


def test_step_alpha_pin_rejects_planted_mistakes():
    """Plausible slips in the step size (planted in a copy of the oracle's
    function, on the CPU) each move alpha off the top eigenvalue."""
    def scaled(A, B, g, lam, t):
        return 1.01 * oracle.step_alpha(A, B, g, lam, t)

    def lam_not_over_t(A, B, g, lam, t):
        return oracle.step_alpha(A, B, g, lam, 1)

    def sum_not_max(A, B, g, lam, t):
        Gc = np.diag(g)
        MB = Gc.conj().T @ (B.conj().T @ B) @ Gc
        MA = Gc.conj().T @ (A.conj().T @ A) @ Gc
        return lam / t + oracle.gershgorin(MB) + oracle.gershgorin(MA)

    for bad in (scaled, lam_not_over_t, sum_not_max):
        alpha, top, _ = _alpha_pin_case(0, bad)
        assert abs(alpha - top) > 1e-6 * top, bad.__name__


def test_step_alpha_through_the_push_at_t3():
    """The alpha a push reports is the same exact value (the push's own gamma)."""
    rng = _rng(47)
    n1, n2, R = 7, 6, 3
    A = _orthogonal_columns(rng, n1, [1.7, 0.6, 1.1])
    B = _orthogonal_columns(rng, n2, [0.5, 1.3, 0.9])
    lam = 0.9
    o = oracle.TslOracle(n1, n2, R, lam, A, B)
    o.t, o.abar = 2, 5.0                                  # the state after two frames
    s = o.push_points(np.ones((n1, n2), bool), _cn(rng, (n1, n2)))
    assert s.t == 3
    Fl, Fr = o.Fl, o.Fr
    oi, oj = np.nonzero(np.ones((n1, n2), bool))
    top = 0.0
    for wrt in ("A", "B"):
        Lop = _block_operator(A, B, s.gamma, oi, oj, Fl, Fr, wrt)
        top = max(top, float(np.linalg.eigvalsh(Lop.conj().T @ Lop).max()) + lam / 3)
    assert abs(s.alpha - top) <= 1e-12 * top
    assert abs(s.alpha_bar - (5.0 + top)) <= 1e-12 * (5.0 + top)
    assert abs(s.mu - 1.0 / (5.0 + top)) <= 1e-12 / (5.0 + top)


def test_mm_majorized_cost_never_increases():
    c = I.config1(T=8)
    o = oracle.TslOracle(c["n1"], c["n2"], c["r"], 0.1, c["A0"], c["B0"])
    for fr in c["frames"]:
        A0, B0 = o.A.copy(), o.B.copy()
        s = o.push_points(fr.mask, fr.y)
        f = lambda a, b: oracle.instantaneous_cost(a, b, s.gamma, s.oi, s.oj, s.y, 0.1, s.t, o.Fl, o.Fr)
        f0 = f(A0, B0)
        for new, grad_at in (("A", (s.A, B0)), ("B", (A0, s.B))):
            delta = (s.A - A0) if new == "A" else (s.B - B0)
            grad = -delta / s.mu
            surrogate = f0 + np.vdot(grad, delta).real + 0.5 * s.alpha * np.vdot(delta, delta).real
            f_new = f(*grad_at)
            assert f_new <= surrogate * (1 + 1e-12) + 1e-12
            assert surrogate <= f0 * (1 + 1e-12) + 1e-12


def test_recursion_equals_weighted_sum_of_mm_minimisers():
    rng, n1, n2, R, A, B = _tiny_state(11)
    lam = 0.25
    o = oracle.TslOracle(n1, n2, R, lam, A, B)
    Fl, Fr = o.Fl, o.Fr
    acc, abar = np.zeros_like(o.A), 0.0
    for _ in range(4):
        A_prev, B_prev = o.A.copy(), o.B.copy()
        mask = rng.random((n1, n2)) < 0.6
        s = o.push_points(mask, _cn(rng, (n1, n2)))
        g = _explicit_gradient(A_prev, B_prev, s.gamma, s.oi, s.oj, s.y, lam, s.t, Fl, Fr, "A")
        acc += s.alpha * (A_prev - g / s.alpha)
        abar += s.alpha
        assert np.allclose(o.A, acc / abar, atol=1e-12)        # A[t] = (1/abar_t) sum alpha_tau {...}


# ----------------------------------------------------------------- whole-step special cases
def test_exact_recovery_noiseless_full_sampling_lambda0():
    c = I.config1(T=4, exact=True)
    A, B, G = c["truth"]
    o = oracle.TslOracle(c["n1"], c["n2"], c["r"], 0.0, A, B)
    for t, fr in enumerate(c["frames"]):
        # the stored frames are complex64; take the FP64 k-space of the truth here
        s = o.push_points(fr.mask, np.fft.fft2(fr.truth, norm="ortho"))
        assert _nr(s.gamma, G[t]) < 1e-11
        assert np.max(np.abs(s.e)) < 1e-10
        assert _nr(s.A, A) < 1e-12 and _nr(s.B, B) < 1e-12
        assert _nr(s.X, fr.truth) < 1e-11


def test_recovery_from_perturbed_factors_noiseless_full_sampling():
    """Started off the truth (true factors plus CN(0, 1e-4) noise), lambda = 0,
    every point sampled, one noiseless frame pushed repeatedly: the S2 update
    must move the factors towards the data.  The fit residual ||y - Phi gamma||
    after each frame's ridge solve never increases and falls at least fourfold
    over 30 frames, and the output frame approaches the truth."""
    c = I.config1(T=1, exact=True, perturb=1e-2)
    o = oracle.TslOracle(c["n1"], c["n2"], c["r"], 0.0, c["A0"], c["B0"])
    truth = c["frames"][0].truth
    Y = np.fft.fft2(truth, norm="ortho")
    full = np.ones((c["n1"], c["n2"]), bool)
    res, err = [], []
    for _ in range(30):
        s = o.push_points(full, Y)
        res.append(float(np.linalg.norm(s.e)))
        err.append(_nr(s.X, truth))
    res = np.array(res)
    assert res[0] > 1e-3                                 # the start is really off the truth
    assert np.all(np.diff(res) <= 1e-12 * res[0])
    assert res[-1] < 0.25 * res[0]
    assert err[-1] < 0.5 * err[0]


def test_exact_data_with_lambda_gives_shrunk_closed_form():
    c = I.config1(T=1, exact=True)
    A, B, G = c["truth"]
    lam = 3.0
    o = oracle.TslOracle(c["n1"], c["n2"], c["r"], lam, A, B)
    s = o.push_points(c["frames"][0].mask, np.fft.fft2(c["frames"][0].truth, norm="ortho"))
    P = (A.conj().T @ A) * (B.conj().T @ B)          # Phi^H Phi for the full mask (Schur product)
    assert _nr(s.gamma, np.linalg.solve(P + lam * np.eye(c["r"]), P @ G[0])) < 1e-10


def test_empty_mask_is_pure_shrink():
    rng, n1, n2, R, A, B = _tiny_state(12)
    o = oracle.TslOracle(n1, n2, R, 0.5, A, B)
    s = o.push_lines(np.zeros(0, np.int32), np.zeros((0, n2)))
    assert np.all(s.gamma == 0) and np.allclose(s.A, s.shrink * A) and np.allclose(s.B, s.shrink * B)
    assert s.alpha == pytest.approx(0.5)


def test_lines_equal_points_on_full_rows():
    rng, n1, n2, R, A, B = _tiny_state(13, n1=16, n2=12, R=4)
    rows = np.array([0, 3, 4, 9, 15], np.int32)
    Y = _cn(rng, (n1, n2))
    mask = np.zeros((n1, n2), bool); mask[rows] = True
    a = oracle.TslOracle(n1, n2, R, 0.2, A, B).push_lines(rows, Y[rows])
    b = oracle.TslOracle(n1, n2, R, 0.2, A, B).push_points(mask, Y)
    assert np.allclose(a.X, b.X, atol=1e-13) and np.allclose(a.gamma, b.gamma, atol=1e-13)


@pytest.mark.parametrize("kind", ["lines", "points"])
def test_image_domain_step_equals_kspace_interpolation_step(kind):
    rng = _rng(14)
    n1, n2, R, lam = 20, 16, 5, 0.15
    A0, B0 = 0.3 * _cn(rng, (n1, R)), 0.3 * _cn(rng, (n2, R))
    Fl, Fr = oracle.dft_matrix(n1), oracle.dft_matrix(n2)
    img = oracle.TslOracle(n1, n2, R, lam, A0, B0)
    ksp = oracle.KspaceOracle(n1, n2, R, lam, Fl @ A0, Fr @ B0)
    for t in range(6):
        Y = _cn(rng, (n1, n2))
        if kind == "lines":
            rows = np.sort(rng.choice(n1, 7, replace=False)).astype(np.int32)
            a, b = img.push_lines(rows, Y[rows]), ksp.push_lines(rows, Y[rows])
        else:
            mask = rng.random((n1, n2)) < 0.3
            a, b = img.push_points(mask, Y), ksp.push_points(mask, Y)
        assert _nr(a.gamma, b.gamma) < 1e-11
        assert _nr(Fl @ a.A, b.alpha_f) < 1e-11
        assert _nr(Fr @ a.B, b.beta_f) < 1e-11
        assert _nr(a.X, oracle.ifft2_unitary(b.Xk)) < 1e-11


# ----------------------------------------------------------------- sampler (Sec. V, Sec. VI-C)
def test_philox_known_answer_vectors():
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for w in rows:
        v = [int(x, 16) for x in w]
        assert oracle.philox4x64_10(v[0:4], v[4:6]) == v[6:10]


def test_philox_matches_numpy_bit_generator():
    # numpy's Philox advances its counter before the first block: block c+1 first.
    key = [0x1234567890ABCDEF, 42]
    for ctr in ([0, 0, 0, 0], [7, 3, 0, 0], [2**64 - 1, 5, 0, 0]):
        bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
        raw = [int(x) for x in bg.random_raw(4)]
        nxt = list(ctr)
        nxt[0] = (nxt[0] + 1) % 2**64
        if nxt[0] == 0:
            nxt[1] += 1
        assert oracle.philox4x64_10(nxt, key) == raw


def test_scores_sum_to_one_and_line_score_is_the_marginal():
    rng = _rng(15)
    n1, n2, R = 24, 18, 5
    Ah, Bh = _cn(rng, (n1, R)), _cn(rng, (n2, R))
    s2 = point_scores(Ah, Bh)
    s1 = oracle.line_scores(Ah, n2)
    assert abs(s2.sum() - 1.0) < 1e-13 and abs(s1.sum() - 1.0) < 1e-13
    assert np.all(s2 > 0)
    assert np.allclose(s2.sum(axis=1), s1, atol=1e-15)      # Sec. VI-C marginal of eq. 13
    _, prefix = oracle.line_weights_prefix(Ah, n2)
    assert abs(prefix[-1] - R * (n1 + n2)) < 1e-11 * R * (n1 + n2)


def test_uniform_factor_rows_give_uniform_scores():
    n1, R = 16, 4
    F = oracle.dft_matrix(n1)[:, :R]           # every entry has |.|^2 = 1/n1
    s = oracle.line_scores(F.astype(np.complex64), 10)
    assert np.allclose(s, 1.0 / n1, atol=1e-7)


def test_zero_column_is_skipped():
    rng = _rng(16)
    Ah = _cn(rng, (12, 3)); Ah[:, 1] = 0
    s = oracle.line_scores(Ah, 7)
    assert np.all(np.isfinite(s)) and abs(s.sum() - 1) < 1e-13


def test_expected_sample_count_and_draw_frequencies():
    rng = _rng(17)
    n1, n2, R, K = 32, 20, 4, 10
    Ah = _cn(rng, (n1, R)) * np.exp(-0.15 * np.arange(n1))[:, None]
    s = oracle.line_scores(Ah, n2)
    counts, freq = [], np.zeros(n1)
    n_streams = 3000
    for stream in range(n_streams):
        rows, draws = oracle.draw_lines(Ah, n2, K, seed=99, stream=stream, t=1)
        counts.append(rows.size)
        np.add.at(freq, draws, 1)
    counts = np.array(counts, float)
    mean, se = counts.mean(), counts.std(ddof=1) / np.sqrt(n_streams)
    assert abs(mean - expected_count(s, K)) < 2.58 * se + 1e-9     # 99 % interval (Sec. V-B)
    exp = s * K * n_streams
    chi2 = float(np.sum((freq - exp) ** 2 / exp))
    import scipy.stats
    assert chi2 < scipy.stats.chi2.ppf(1 - 1e-4, n1 - 1)


def test_draws_are_deterministic_sorted_unique():
    rng = _rng(18)
    Ah = _cn(rng, (40, 6)).astype(np.complex64)
    r1, d1 = oracle.draw_lines(Ah, 33, 12, seed=5, stream=2, t=9)
    r2, d2 = oracle.draw_lines(Ah, 33, 12, seed=5, stream=2, t=9)
    assert np.array_equal(r1, r2) and np.array_equal(d1, d2)
    assert np.all(np.diff(r1) > 0) and r1.size <= 12 and set(d1.tolist()) == set(r1.tolist())
    d_other = [oracle.draw_lines(Ah, 33, 12, seed=5, stream=2, t=t)[1] for t in (10, 11, 12)]
    assert any(not np.array_equal(d1, d) for d in d_other)      # the counter carries t


# ----------------------------------------------------------------- regression fixture
def test_oracle_matches_its_committed_fixture():
    import json
    with open(os.path.join(GOLDEN, "oracle_config1_first_frames.json")) as fh:
        gold = json.load(fh)
    c = I.config1(T=len(gold["gamma"]))
    o = oracle.TslOracle(c["n1"], c["n2"], c["r"], 0.1, c["A0"], c["B0"])
    for t, fr in enumerate(c["frames"]):
        s = o.push_points(fr.mask, fr.y)
        g = np.array(gold["gamma"][t][0]) + 1j * np.array(gold["gamma"][t][1])
        assert _nr(s.gamma, g) < 1e-12
        assert abs(s.alpha_bar - gold["alpha_bar"][t]) < 1e-9 * gold["alpha_bar"][t]


def test_blocked_sums_follow_the_stated_order():
    from oracle.sampler import SUM_BLOCK, blocked_prefix, blocked_sum
    assert SUM_BLOCK == 16
    # integer-valued terms: every order is exact, so the sum and the prefix are the exact ones
    rng = _rng(19)
    x = rng.integers(0, 1000, size=77).astype(np.float64)
    assert blocked_sum(x) == float(x.sum())
    assert np.array_equal(blocked_prefix(x), np.cumsum(x))
    # an order-sensitive case: 1 followed by 31 terms of 2^-53.  Added one by one
    # each small term is lost against 1; in blocks of 16 the second block's
    # sixteen terms meet first (2^-49) and survive
    y = np.array([1.0] + [2.0 ** -53] * 31)
    seq = 0.0
    for v in y:
        seq = seq + v
    assert seq == 1.0
    assert blocked_sum(y) == 1.0 + 2.0 ** -49
    p = blocked_prefix(y)
    assert p[15] == 1.0 and p[16] == 1.0 and p[31] == 1.0 + 2.0 ** -49
    assert p[-1] == blocked_sum(y)
    # within one block the prefix is the sequential one
    z = rng.random(SUM_BLOCK)
    seq_p, run = [], 0.0
    for v in z:
        run = run + v
        seq_p.append(run)
    assert np.array_equal(blocked_prefix(z), np.array(seq_p))
    # the sum over columns of a 2-D array goes along the leading axis
    m = rng.random((40, 3))
    assert np.array_equal(blocked_sum(m), np.array([blocked_sum(m[:, j]) for j in range(3)]))


# ---------------------------------------------------------------------------- Gram conditioning figure
def test_pivot_ratio_is_kappa_for_a_diagonal_gram_and_bounds_it_otherwise():
    rng = _rng(90)
    d = np.array([3.0, 0.25, 7.5, 1.0])
    assert abs(oracle.gram_pivot_ratio(np.diag(d).astype(complex)) - 30.0) <= 1e-12 * 30.0
    for _ in range(20):
        M = _cn(rng, (6, 4))
        G = M.conj().T @ M + 0.1 * np.eye(4)
        ev = np.linalg.eigvalsh(G)
        assert oracle.gram_pivot_ratio(G) <= ev[-1] / ev[0] * (1 + 1e-12)


def test_pivot_ratio_two_by_two_closed_form():
    """G = [[a, b], [conj(b), c]]: the pivots are a and c - |b|^2 / a."""
    a, b, c = 2.0, 0.7 - 0.4j, 1.3
    G = np.array([[a, b], [np.conj(b), c]])
    d2 = c - abs(b) ** 2 / a
    want = max(a, d2) / min(a, d2)
    assert abs(oracle.gram_pivot_ratio(G) - want) <= 1e-12 * want


# ---------------------------------------------------------------------------- batch passes (Sec. VI-D)
def _epoch_case(E, lam=1e-3):
    c = I.config1(T=6, exact=True, perturb=3e-2)
    frames = [("points", fr.mask, fr.y) for fr in c["frames"]]
    rng = _rng(60)
    order = [np.arange(6)] + [rng.permutation(6) for _ in range(E - 1)]
    o = oracle.TslOracle(c["n1"], c["n2"], c["r"], lam, c["A0"], c["B0"])
    last = oracle.epochs(o, frames, order)
    err = float(np.mean([_nr(s.X, fr.truth) ** 2 for s, fr in zip(last, c["frames"])]))
    return o, last, err, order, frames, c


def test_epochs_carry_the_subspace_from_pass_to_pass():
    """Noiseless rank-R frames, every point sampled, started off the true
    factors: later passes start from what earlier ones learnt, so the mean NMSE
    of the frames' last reconstructions falls with the number of passes (a
    restart at every pass would leave it where one pass leaves it)."""
    errs = [_epoch_case(E)[2] for E in (1, 2, 4)]
    assert errs[1] < 0.9 * errs[0] and errs[2] < 0.9 * errs[1], errs


def test_epochs_are_the_pushes_in_pass_order():
    """Two passes in one call equal the same visits pushed one by one, and t
    counts every visit (12 after two passes over six frames)."""
    o, last, _, order, frames, c = _epoch_case(2)
    ref = oracle.TslOracle(c["n1"], c["n2"], c["r"], 1e-3, c["A0"], c["B0"])
    for perm in order:
        for v in perm:
            s = ref.push_points(frames[v][1], frames[v][2])
    assert o.t == 12 and ref.t == 12
    assert np.array_equal(o.A, ref.A) and np.array_equal(o.B, ref.B) and o.abar == ref.abar
    assert np.array_equal(last[order[-1][-1]].X, s.X)


def test_epochs_reject_an_order_that_is_not_a_permutation():
    c = I.config1(T=3)
    frames = [("points", fr.mask, fr.y) for fr in c["frames"]]
    o = oracle.TslOracle(c["n1"], c["n2"], c["r"], 0.1, c["A0"], c["B0"])
    with pytest.raises(ValueError):
        oracle.epochs(o, frames, [[0, 1, 1]])


# ---------------------------------------------------------------------------- point sampling (eq. 13)
def test_point_mixture_is_the_score_of_eq13():
    """The two-component mixture the point draw uses assigns every entry the
    probability eq. 13 gives it (and the probabilities sum to one); the mixture
    weights swapped would not."""
    rng = _rng(71)
    Ah, Bh = _cn(rng, (9, 3)), _cn(rng, (7, 3))
    s13 = oracle.point_scores(Ah, Bh)
    mix = oracle.point_draw_probabilities(Ah, Bh)
    assert abs(s13.sum() - 1.0) < 1e-13 and abs(mix.sum() - 1.0) < 1e-13
    assert np.max(np.abs(mix - s13)) < 1e-15
    qa, pa, qb, pb = oracle.point_weights_prefix(Ah, Bh)
    n1, n2 = 9, 7
    swapped = (n1 / (n1 + n2)) * (qa / pa[-1])[:, None] / n2 + (n2 / (n1 + n2)) * (qb / pb[-1])[None, :] / n1
    assert np.max(np.abs(swapped - s13)) > 1e-3


def test_point_draws_follow_eq13_and_expected_count():
    rng = _rng(72)
    n1, n2, R, K = 6, 5, 2, 12
    Ah = _cn(rng, (n1, R)) * np.exp(-0.4 * np.arange(n1))[:, None]
    Bh = _cn(rng, (n2, R)) * np.exp(-0.3 * np.arange(n2))[:, None]
    s = oracle.point_scores(Ah, Bh)
    freq, counts = np.zeros((n1, n2)), []
    n_frames = 1500
    for t in range(1, n_frames + 1):
        mask, draws = oracle.draw_points(Ah, Bh, K, seed=3, stream=1, t=t)
        counts.append(int(mask.sum()))
        np.add.at(freq, (draws[:, 0], draws[:, 1]), 1)
        assert set(map(tuple, draws.tolist())) == set(zip(*np.nonzero(mask)))
    exp = s * K * n_frames
    chi2 = float(np.sum((freq - exp) ** 2 / exp))
    import scipy.stats
    assert chi2 < scipy.stats.chi2.ppf(1 - 1e-4, n1 * n2 - 1)
    counts = np.array(counts, float)
    mean, se = counts.mean(), counts.std(ddof=1) / np.sqrt(n_frames)
    assert abs(mean - oracle.expected_count(s, K)) < 2.58 * se + 1e-9     # E|Omega| of Sec. V-B


def test_point_draws_skip_a_zero_column():
    rng = _rng(73)
    Ah, Bh = _cn(rng, (8, 3)), _cn(rng, (6, 3))
    Ah[:, 1] = 0
    mix = oracle.point_draw_probabilities(Ah, Bh)
    assert np.all(np.isfinite(mix)) and abs(mix.sum() - 1.0) < 1e-13
    mask, draws = oracle.draw_points(Ah.astype(np.complex64), Bh.astype(np.complex64), 20, 1, 2, 3)
    assert mask.sum() >= 1 and np.all(draws >= 0) and np.all(draws[:, 0] < 8) and np.all(draws[:, 1] < 6)


# ---------------------------------------------------------------------------- several coils (Sec. IV-B)
def _coil_case(seed, n1=6, n2=5, R=2, C=3):
    rng = _rng(80 + seed)
    A, B = _cn(rng, (n1, R)), _cn(rng, (n2, R))
    H = _cn(rng, (C, n1, n2))
    return rng, A, B, H


def test_one_all_ones_coil_is_the_single_coil_step():
    c = I.config2(T=4, n1=16, n2=12, r=3, accel=2, t_warm=1)
    a = oracle.TslOracle(16, 12, 3, 0.05, c["A0"], c["B0"])
    b = oracle.CoilOracle(16, 12, 3, 0.05, c["A0"], c["B0"], np.ones((1, 16, 12)))
    for fr in c["frames"]:
        sa = a.push_lines(fr.rows, fr.y)
        sb = b.push_lines(fr.rows, fr.y[None])
        for k in ("gamma", "A", "B", "X"):
            assert _nr(getattr(sb, k), getattr(sa, k)) < 1e-12, k
        assert abs(sb.alpha - sa.alpha) < 1e-12 * sa.alpha


def test_coil_back_projection_is_the_explicit_sketch_sum():
    """Theta = sum_c sum_l e_c^l conj(W_c^l) with W_c^(i,j) = H_c .* F(e_i e_j^T)
    (Sec. IV-B), summed matrix by matrix, equals sum_c conj(H_c) .* F^{-1}(Xi_c)."""
    rng, A, B, H = _coil_case(1)
    n1, n2, C = 6, 5, 3
    o = oracle.CoilOracle(n1, n2, 2, 0.2, A, B, H)
    rows = np.array([0, 2, 5], dtype=np.int32)
    s = o.push_lines(rows, _cn(rng, (C, 3, n2)))
    Fl, Fr = oracle.dft_matrix(n1), oracle.dft_matrix(n2)
    Theta = np.zeros((n1, n2), complex)
    for c in range(C):
        for q, i in enumerate(rows):
            for j in range(n2):
                E = np.zeros((n1, n2)); E[i, j] = 1.0
                W = H[c] * (Fl @ E @ Fr)
                Theta += s.e[c, q, j] * np.conj(W)
    assert _nr(s.Theta, Theta) < 1e-12


def test_coil_regression_matrix_is_the_coil_weighted_synthesis():
    """Phi gamma read at the samples equals F(H_c .* A diag(gamma) B^T) at the
    sampled rows (linearity), coil by coil."""
    rng, A, B, H = _coil_case(2)
    Fl, Fr = oracle.dft_matrix(6), oracle.dft_matrix(5)
    rows = np.array([1, 3, 4])
    g = _cn(rng, 2)
    Phi = oracle.coil_regression_matrix(A, B, H, rows, Fl, Fr)
    X = A @ np.diag(g) @ B.T
    want = np.concatenate([(Fl @ (H[c] * X) @ Fr)[rows, :].reshape(-1) for c in range(3)])
    assert _nr(Phi @ g, want) < 1e-13


def test_coil_update_is_the_gradient_by_finite_differences():
    """(A[t-1] - A[t]) / mu_t is the gradient of the several-coil cost
    1/2 sum_c ||y_c - F(H_c .* A diag(gamma) B^T)_S||^2 + lambda/(2t) ||A||^2."""
    rng, A, B, H = _coil_case(3)
    lam = 0.3
    o = oracle.CoilOracle(6, 5, 2, lam, A, B, H)
    rows = np.array([0, 1, 4], dtype=np.int32)
    Y = _cn(rng, (3, 3, 5))
    s = o.push_lines(rows, Y)
    Fl, Fr = o.Fl, o.Fr
    gA, gB = (A - s.A) / s.mu, (B - s.B) / s.mu

    def cost(a, b):
        X = a @ np.diag(s.gamma) @ b.T
        r = np.concatenate([(Y[c] - (Fl @ (H[c] * X) @ Fr)[rows, :]).reshape(-1) for c in range(3)])
        return 0.5 * np.vdot(r, r).real + lam / (2 * s.t) * (np.vdot(a, a).real + np.vdot(b, b).real)

    h = 1e-6
    for _ in range(3):
        E = _cn(rng, A.shape)
        fd = (cost(A + h * E, B) - cost(A - h * E, B)) / (2 * h)
        assert abs(fd - np.vdot(gA, E).real) < 1e-6 * max(1.0, abs(fd))
        E = _cn(rng, B.shape)
        fd = (cost(A, B + h * E) - cost(A, B - h * E)) / (2 * h)
        assert abs(fd - np.vdot(gB, E).real) < 1e-6 * max(1.0, abs(fd))


def test_coil_step_size_bounds_the_block_hessian_and_is_exact_for_constant_maps():
    rng, A, B, H = _coil_case(4)
    n1, n2, C, R = 6, 5, 3, 2
    Fl, Fr = oracle.dft_matrix(n1), oracle.dft_matrix(n2)
    g = _cn(rng, R)
    lam, t = 0.4, 2

    def top_eig(A, B, H, rows, wrt):
        n = A.shape[0] if wrt == "A" else B.shape[0]
        cols = []
        for r in range(R):
            for m in range(n):
                D = np.zeros((n, R), complex); D[m, r] = 1.0
                X = (D * g) @ B.T if wrt == "A" else (A * g) @ D.T
                cols.append(np.concatenate([(Fl @ (H[c] * X) @ Fr)[rows, :].reshape(-1) for c in range(len(H))]))
        L = np.array(cols).T
        return float(np.linalg.eigvalsh(L.conj().T @ L).max())

    def alpha(A, B, H):
        return lam / t + oracle.coil_gain(H) * oracle.step_alpha(A, B, g, 0.0, t)

    rows = np.array([0, 2, 3])
    for wrt in ("A", "B"):
        assert top_eig(A, B, H, rows, wrt) + lam / t <= alpha(A, B, H) * (1 + 1e-12)
    # constant maps (H_c = eta_c everywhere), orthogonal factor columns, every row:
    # the bound is the top eigenvalue of the factor-block Hessians
    Ao = _orthogonal_columns(rng, n1, [1.4, 0.7])
    Bo = _orthogonal_columns(rng, n2, [0.6, 1.2])
    eta = _cn(rng, C)
    Hc = eta[:, None, None] * np.ones((C, n1, n2))
    full = np.arange(n1)
    top = max(top_eig(Ao, Bo, Hc, full, w) for w in ("A", "B")) + lam / t
    assert abs(alpha(Ao, Bo, Hc) - top) <= 1e-12 * top


def test_coil_exact_recovery_noiseless_full_sampling_lambda0():
    c = I.config1(T=3, n=16, r=3, exact=True)
    A, B, G = c["truth"]
    rng = _rng(85)
    H = I.coil_maps(16, 16, 4, rng).astype(np.complex128)
    o = oracle.CoilOracle(16, 16, 3, 0.0, A, B, H)
    rows = np.arange(16)
    for k, fr in enumerate(c["frames"]):
        Y = np.stack([(o.Fl @ (H[q] * fr.truth) @ o.Fr) for q in range(4)])
        s = o.push_lines(rows, Y)
        assert _nr(s.gamma, G[k]) < 1e-11
        assert _nr(s.X, fr.truth) < 1e-11
        assert _nr(s.A, A) < 1e-12 and _nr(s.B, B) < 1e-12


def test_coil_maps_are_sum_of_squares_normalised():
    H = I.coil_maps(24, 20, 6, _rng(86)).astype(np.complex128)
    assert np.allclose(np.sum(np.abs(H) ** 2, axis=0), 1.0, atol=1e-6)
    assert abs(oracle.coil_gain(H) - 1.0) < 1e-6
