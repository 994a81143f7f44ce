"""GPU parity of the HIP step against the FP64 oracle, through the C ABI.

Tolerance: relative NRMSE ||x_gpu - x_oracle|| / ||x_oracle|| <= 1e-4 per frame for
X_t, A[t], B[t] and gamma_t (complex64 frame path, FP64 R x R statistics, against
an all-FP64 oracle).  Integer outputs (sampled rows) must match bit for bit.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1609_04104_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_04104_amd import tsl
    tsl.lib()
    return tsl


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def nr(a, b):
    b = np.asarray(b)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - b) / (den if den > 0 else 1.0))


def cn(rng, shape, var=1.0):
    return (rng.normal(0, np.sqrt(var / 2), shape) + 1j * rng.normal(0, np.sqrt(var / 2), shape))


class Outs:
    def __init__(self, n1, n2, r):
        self.X = torch.zeros(n1, n2, dtype=torch.complex64, device="cuda")
        self.A = torch.zeros(n1, r, dtype=torch.complex64, device="cuda")
        self.B = torch.zeros(n2, r, dtype=torch.complex64, device="cuda")
        self.g = torch.zeros(r, dtype=torch.complex64, device="cuda")

    def kw(self):
        return dict(X_out=self.X, A_out=self.A, B_out=self.B, gamma_out=self.g)


def compare_step(o, s, tag):
    errs = {"X": nr(host(o.X), s.X), "A": nr(host(o.A), s.A), "B": nr(host(o.B), s.B),
            "gamma": nr(host(o.g), s.gamma)}
    bad = {k: v for k, v in errs.items() if not v <= TOL}
    assert not bad, f"{tag}: {errs}"
    return errs


# ---------------------------------------------------------------------------- a5 / a7
FFT_SHAPES = [(8, 16), (16, 24), (24, 32), (32, 40), (40, 48), (48, 64), (64, 80), (80, 96), (96, 100),
              (100, 120), (120, 128), (128, 144), (144, 160), (160, 192), (192, 200), (200, 240),
              (240, 256), (256, 288), (288, 320), (320, 384), (384, 400), (400, 480), (480, 512), (512, 8)]


@pytest.mark.parametrize("n1,n2", FFT_SHAPES)
def test_fft2_matches_dense_dft(T, n1, n2):
    print(f"fft2 {n1}x{n2}", flush=True)
    rng = np.random.default_rng(n1 * 1000 + n2)
    x = cn(rng, (2, n1, n2)).astype(np.complex64)
    Fl, Fr = oracle.dft_matrix(n1), oracle.dft_matrix(n2)
    ref = np.stack([oracle.fft2_unitary(x[b].astype(np.complex128), Fl, Fr) for b in range(2)])
    got = host(T.fft2(dev(x)))
    assert nr(got, ref) < 2e-6
    back = host(T.fft2(dev(got), inverse=True))
    assert nr(back, x) < 4e-6
    # in place
    xd = dev(x)
    T.fft2(xd, out=xd)
    assert nr(host(xd), ref) < 2e-6


# ---------------------------------------------------------------------------- one step
def _random_state(n1, n2, r, seed):
    rng = np.random.default_rng(seed)
    A0 = cn(rng, (n1, r), 1.0 / n1).astype(np.complex64)
    B0 = cn(rng, (n2, r), 1.0 / n2).astype(np.complex64)
    return rng, A0, B0


@pytest.mark.parametrize("n1,n2,r,nrows", [(64, 64, 8, 20), (256, 256, 32, 32), (120, 200, 5, 37),
                                           (192, 160, 16, 1), (128, 128, 64, 128), (160, 320, 24, 11),
                                           (384, 96, 48, 200), (16, 8, 3, 16)])
@pytest.mark.parametrize("route", ["kspace", "frame"])
def test_one_line_step_matches_oracle(T, n1, n2, r, nrows, route):
    print(f"one step lines {n1}x{n2} r={r} rows={nrows} route={route}", flush=True)
    rng, A0, B0 = _random_state(n1, n2, r, n1 + 7 * n2 + r)
    rows = np.sort(rng.choice(n1, nrows, replace=False)).astype(np.int32)
    Y = cn(rng, (nrows, n2), 1.0 / (n1 * n2) * 50).astype(np.complex64)
    lam = 0.05
    ora = oracle.TslOracle(n1, n2, r, lam, A0, B0)
    seq = T.Sequence(n1, n2, r, lam, dev(A0), dev(B0), route=route)
    o = Outs(n1, n2, r)
    for t in range(3):
        s = ora.push_lines(rows, Y)
        seq.push_lines(dev(rows), dev(Y), **o.kw())
        compare_step(o, s, f"t={t + 1}")
        Ah = torch.zeros(n1, r, dtype=torch.complex64, device="cuda")
        Bh = torch.zeros(n2, r, dtype=torch.complex64, device="cuda")
        seq.factors(Ahat=Ah, Bhat=Bh)
        Ah_o, Bh_o = ora.kspace_factors()
        assert nr(host(Ah), Ah_o) < TOL and nr(host(Bh), Bh_o) < TOL
    assert seq.status() == 0
    seq.close()


@pytest.mark.parametrize("n1,n2,r,frac", [(64, 64, 8, 0.25), (40, 48, 6, 0.5), (128, 120, 12, 0.1)])
def test_one_point_step_matches_oracle(T, n1, n2, r, frac):
    print(f"one step points {n1}x{n2} r={r}", flush=True)
    rng, A0, B0 = _random_state(n1, n2, r, 3 * n1 + n2)
    lam = 0.1
    ora = oracle.TslOracle(n1, n2, r, lam, A0, B0)
    seq = T.Sequence(n1, n2, r, lam, dev(A0), dev(B0))
    o = Outs(n1, n2, r)
    for t in range(3):
        mask = rng.random((n1, n2)) < frac
        Y = np.where(mask, cn(rng, (n1, n2), 1.0 / (n1 * n2) * 20), 0).astype(np.complex64)
        s = ora.push_points(mask, Y)
        seq.push_points(dev(mask.astype(np.uint8)), dev(Y), **o.kw())
        compare_step(o, s, f"t={t + 1}")
    seq.close()


# ---------------------------------------------------------------------------- trajectories
def test_config1_trajectory_points(T):
    print("config 1 trajectory", flush=True)
    c = I.config1()
    n, r = c["n1"], c["r"]
    ora = oracle.TslOracle(n, n, r, 0.1, c["A0"], c["B0"])
    seq = T.Sequence(n, n, r, 0.1, dev(c["A0"]), dev(c["B0"]))
    o = Outs(n, n, r)
    worst = {}
    for t, fr in enumerate(c["frames"]):
        s = ora.push_points(fr.mask, fr.y)
        seq.push_points(dev(fr.mask.astype(np.uint8)), dev(fr.y), **o.kw())
        e = compare_step(o, s, f"t={t + 1}")
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0), v)
    print("config 1 worst NRMSE", worst, flush=True)
    seq.close()


def test_config1_exact_recovery(T):
    c = I.config1(T=3, exact=True)
    n, r = c["n1"], c["r"]
    A, B, G = c["truth"]
    seq = T.Sequence(n, n, r, 0.0, dev(c["A0"]), dev(c["B0"]), allow_lambda0=True)
    o = Outs(n, n, r)
    for t, fr in enumerate(c["frames"]):
        seq.push_points(dev(fr.mask.astype(np.uint8)), dev(fr.y), **o.kw())
        assert nr(host(o.g), G[t]) < 1e-5
        assert nr(host(o.X), fr.truth) < 1e-5
        assert nr(host(o.A), A) < 1e-5
    seq.close()


def test_recovery_from_perturbed_factors_matches_oracle(T):
    """The oracle's recovery pin (true factors plus CN(0, 1e-4), lambda = 0,
    every point sampled, one noiseless frame pushed 30 times) on the device:
    per-frame parity, and the residual falls as the oracle's does."""
    print("recovery from perturbed factors", flush=True)
    c = I.config1(T=1, exact=True, perturb=1e-2)
    n, r = c["n1"], c["r"]
    truth = c["frames"][0].truth
    Y = np.fft.fft2(truth, norm="ortho").astype(np.complex64)     # both sides read the same samples
    full = np.ones((n, n), bool)
    ora = oracle.TslOracle(n, n, r, 0.0, c["A0"], c["B0"])
    seq = T.Sequence(n, n, r, 0.0, dev(c["A0"]), dev(c["B0"]), allow_lambda0=True)
    o = Outs(n, n, r)
    md, yd = dev(full.astype(np.uint8)), dev(Y)
    worst, first, last = 0.0, None, None
    for t in range(30):
        s = ora.push_points(full, Y)
        seq.push_points(md, yd, **o.kw())
        worst = max(worst, max(compare_step(o, s, f"t={t + 1}").values()))
        e = nr(host(o.X), truth)
        first = e if first is None else first
        last = e
    assert seq.status() == 0
    assert last < 0.5 * first
    print(f"recovery worst NRMSE {worst:.2e}, X error {first:.2e} -> {last:.2e}", flush=True)
    seq.close()


@pytest.mark.parametrize("T_frames", [200])
@pytest.mark.parametrize("route", ["kspace", "frame"])
def test_config2_trajectory_lines(T, T_frames, route):
    print(f"config 2 trajectory T={T_frames} route={route}", flush=True)
    c = I.config2(T=T_frames)
    n1, n2, r = c["n1"], c["n2"], c["r"]
    ora = oracle.TslOracle(n1, n2, r, 0.05, c["A0"], c["B0"])
    seq = T.Sequence(n1, n2, r, 0.05, dev(c["A0"]), dev(c["B0"]), route=route)
    o = Outs(n1, n2, r)
    worst = {}
    for t, fr in enumerate(c["frames"]):
        s = ora.push_lines(fr.rows, fr.y)
        seq.push_lines(dev(fr.rows), dev(fr.y), **o.kw())
        e = compare_step(o, s, f"t={t + 1}")
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0), v)
    print(f"config 2 ({route}) worst NRMSE", worst, flush=True)
    seq.close()


# ---------------------------------------------------------------------------- a11
@pytest.mark.parametrize("n1,n2,r,K", [(256, 256, 32, 32), (64, 64, 8, 50), (120, 200, 5, 7), (512, 64, 128, 300)])
def test_sampler_bit_exact_on_device_factors(T, n1, n2, r, K):
    print(f"sampler {n1}x{n2} r={r} K={K}", flush=True)
    rng, A0, B0 = _random_state(n1, n2, r, 11 * n1 + r)
    A0 = (A0 * np.exp(-0.02 * np.arange(n1))[:, None]).astype(np.complex64)
    seed, sid = 1234567, 42
    seq = T.Sequence(n1, n2, r, 0.05, dev(A0), dev(B0), seed=seed, stream_id=sid)
    for t in range(2):
        if t:
            rows = np.sort(rng.choice(n1, max(1, n1 // 8), replace=False)).astype(np.int32)
            seq.push_lines(dev(rows), dev(cn(rng, (rows.size, n2), 1e-3).astype(np.complex64)))
        rows_out = torch.full((K,), -1, dtype=torch.int32, device="cuda")
        n_out = torch.zeros(1, dtype=torch.int32, device="cuda")
        draws = torch.zeros(K, dtype=torch.int32, device="cuda")
        pref = torch.zeros(n1, dtype=torch.float64, device="cuda")
        seq.sample_lines(K, rows_out, n_out, draws, pref)
        Ah = torch.zeros(n1, r, dtype=torch.complex64, device="cuda")
        seq.factors(Ahat=Ah)
        Ah = host(Ah)
        w, prefix = oracle.line_weights_prefix(Ah, n2)
        assert np.array_equal(host(pref), prefix), "weight prefix differs"
        rows_o, draws_o = oracle.draw_lines(Ah, n2, K, seed, sid, t + 1)
        assert np.array_equal(host(draws), draws_o)
        n = int(host(n_out)[0])
        assert n == rows_o.size and np.array_equal(host(rows_out)[:n], rows_o)
    seq.close()


# ---------------------------------------------------------------------------- errors
def test_device_errors_latch_and_do_not_commit(T):
    n1, n2, r = 64, 48, 4
    rng, A0, B0 = _random_state(n1, n2, r, 99)
    seq = T.Sequence(n1, n2, r, 0.1, dev(A0), dev(B0))
    A = torch.zeros(n1, r, dtype=torch.complex64, device="cuda")
    seq.factors(A=A)
    a0 = host(A).copy()
    Y = dev(cn(rng, (3, n2), 0.01).astype(np.complex64))
    # row out of range
    seq.push_lines(dev(np.array([1, 5, 70], np.int32)), Y)
    assert seq.status() == T.EINVAL
    seq.factors(A=A)
    assert np.array_equal(host(A), a0)
    # later frames are skipped while latched
    seq.push_lines(dev(np.array([1, 5, 7], np.int32)), Y)
    seq.factors(A=A)
    assert np.array_equal(host(A), a0)
    assert seq.status(clear=True) == T.EINVAL
    assert seq.status() == 0
    # not ascending
    seq.push_lines(dev(np.array([5, 1, 7], np.int32)), Y)
    assert seq.status(clear=True) == T.EINVAL
    # NaN sample
    Yn = cn(rng, (3, n2), 0.01).astype(np.complex64)
    Yn[1, 3] = np.nan
    seq.push_lines(dev(np.array([1, 5, 7], np.int32)), dev(Yn))
    assert seq.status(clear=True) == T.ENONFINITE
    seq.factors(A=A)
    assert np.array_equal(host(A), a0)
    # a good frame commits again and matches the oracle started from the same state
    ora = oracle.TslOracle(n1, n2, r, 0.1, A0, B0)
    s = ora.push_lines(np.array([1, 5, 7], np.int32), host(Y))
    o = Outs(n1, n2, r)
    seq.push_lines(dev(np.array([1, 5, 7], np.int32)), Y, **o.kw())
    compare_step(o, s, "after errors")
    seq.close()


def test_lambda0_empty_mask_is_not_pd(T):
    n1, n2, r = 32, 32, 4
    _, A0, B0 = _random_state(n1, n2, r, 5)
    seq = T.Sequence(n1, n2, r, 0.0, dev(A0), dev(B0), allow_lambda0=True)
    seq.push_lines(torch.zeros(0, dtype=torch.int32, device="cuda"),
                   torch.zeros(0, n2, dtype=torch.complex64, device="cuda"))
    assert seq.status(clear=True) == T.ENOTPD
    seq.close()


def test_empty_mask_is_pure_shrink(T):
    n1, n2, r = 32, 40, 4
    _, A0, B0 = _random_state(n1, n2, r, 6)
    ora = oracle.TslOracle(n1, n2, r, 0.5, A0, B0)
    s = ora.push_lines(np.zeros(0, np.int32), np.zeros((0, n2)))
    seq = T.Sequence(n1, n2, r, 0.5, dev(A0), dev(B0))
    o = Outs(n1, n2, r)
    seq.push_lines(torch.zeros(0, dtype=torch.int32, device="cuda"),
                   torch.zeros(0, n2, dtype=torch.complex64, device="cuda"), **o.kw())
    assert np.all(host(o.g) == 0)
    assert nr(host(o.A), s.A) < 1e-6 and nr(host(o.B), s.B) < 1e-6
    seq.close()


def test_argument_errors_are_synchronous(T):
    n1, n2, r = 32, 32, 4
    _, A0, B0 = _random_state(n1, n2, r, 7)
    with pytest.raises(T.TslError) as e:
        T.Sequence(n1, n2, r, 0.0, dev(A0), dev(B0))
    assert e.value.code == T.EINVAL
    with pytest.raises(T.TslError):
        T.Sequence(n1, n2, r, -1.0, dev(A0), dev(B0))
    with pytest.raises(T.TslError):
        T.Sequence(n1, n2, r, 0.1, dev(A0), dev(B0), step_mode="const", mu=0.0)
    seq = T.Sequence(n1, n2, r, 0.1, dev(A0), dev(B0))
    with pytest.raises(T.TslError):
        seq.sample_lines(0, torch.zeros(0, dtype=torch.int32, device="cuda"),
                         torch.zeros(1, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        seq.push_lines(torch.zeros(3, dtype=torch.int32, device="cuda"),
                       torch.zeros(2, n2, dtype=torch.complex64, device="cuda"))
    seq.close()


# ---------------------------------------------------------------------------- batching
def test_step_many_equals_single_pushes_and_oracle(T):
    print("step_many mixed batch", flush=True)
    specs = [(128, 128, 16), (192, 160, 32), (256, 256, 64), (128, 128, 32), (192, 160, 16), (64, 64, 8)]
    rng = np.random.default_rng(77)
    seqs, solo, oras, outs, outs_solo = [], [], [], [], []
    for k, (n1, n2, r) in enumerate(specs):
        _, A0, B0 = _random_state(n1, n2, r, 500 + k)
        route = "frame" if k % 2 else "kspace"     # both routes, and one shape on both (own groups)
        seqs.append(T.Sequence(n1, n2, r, 0.05, dev(A0), dev(B0), route=route))
        solo.append(T.Sequence(n1, n2, r, 0.05, dev(A0), dev(B0), route=route))
        oras.append(oracle.TslOracle(n1, n2, r, 0.05, A0, B0))
        outs.append(Outs(n1, n2, r))
        outs_solo.append(Outs(n1, n2, r))
    for t in range(4):
        frames, keep = [], []
        for k, (n1, n2, r) in enumerate(specs):
            rows = np.sort(rng.choice(n1, n1 // 6, replace=False)).astype(np.int32)
            Y = cn(rng, (rows.size, n2), 1e-3).astype(np.complex64)
            rd, yd = dev(rows), dev(Y)
            keep.append((rd, yd))
            frames.append(seqs[k].frame(rows=rd, y=yd, **outs[k].kw()))
            solo[k].push_lines(rd, yd, **outs_solo[k].kw())
            s = oras[k].push_lines(rows, Y)
            keep.append(s)
        T.step_many(seqs, frames)
        for k in range(len(specs)):
            s = keep[2 * k + 1]
            compare_step(outs[k], s, f"batch seq {k} t={t + 1}")
            assert np.array_equal(host(outs[k].X), host(outs_solo[k].X)), "batched differs from alone"
            assert np.array_equal(host(outs[k].A), host(outs_solo[k].A))
    for s in seqs + solo:
        s.close()


def test_checkpoint_resume_reproduces_frames(T):
    n1, n2, r = 96, 80, 6
    rng, A0, B0 = _random_state(n1, n2, r, 31)
    frames = []
    for t in range(6):
        rows = np.sort(rng.choice(n1, 20, replace=False)).astype(np.int32)
        frames.append((rows, cn(rng, (20, n2), 1e-2).astype(np.complex64)))
    seq = T.Sequence(n1, n2, r, 0.2, dev(A0), dev(B0))
    o = Outs(n1, n2, r)
    for rows, Y in frames[:3]:
        seq.push_lines(dev(rows), dev(Y), **o.kw())
    blob = seq.get_state()
    Xs = []
    for rows, Y in frames[3:]:
        seq.push_lines(dev(rows), dev(Y), **o.kw())
        Xs.append(host(o.X).copy())
    seq.set_state(blob)
    for k, (rows, Y) in enumerate(frames[3:]):
        seq.push_lines(dev(rows), dev(Y), **o.kw())
        assert np.array_equal(host(o.X), Xs[k])
    seq.close()


def test_runs_are_deterministic(T):
    c = I.config1(T=5)
    n, r = c["n1"], c["r"]
    res = []
    for _ in range(2):
        seq = T.Sequence(n, n, r, 0.1, dev(c["A0"]), dev(c["B0"]))
        o = Outs(n, n, r)
        for fr in c["frames"]:
            seq.push_points(dev(fr.mask.astype(np.uint8)), dev(fr.y), **o.kw())
        res.append((host(o.X).copy(), host(o.A).copy()))
        seq.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


# ---------------------------------------------------------------------------- device-drawn rows
def test_config3_device_drawn_rows_match_oracle(T):
    """Informative sampling loop with no host round trip on the device path:
    the GPU draws the rows of frame t+1 from its own F_l A[t]; the oracle's
    sampler on the same (exported) factor must give the same rows bit for bit,
    and the oracle, fed those rows, must track the GPU within the tolerance."""
    print("config 3 device-drawn rows", flush=True)
    Tn = 200
    c = I.config3_kspace(T=Tn)
    n1, n2, r = c["n1"], c["n2"], c["r"]
    K = n1 // 8
    warm = 5
    seq = T.Sequence(n1, n2, r, 0.05, dev(c["A0"]), dev(c["B0"]), seed=77, stream_id=3)
    ora = oracle.TslOracle(n1, n2, r, 0.05, c["A0"], c["B0"])
    Kd = dev(c["kspace"])
    full = torch.arange(n1, dtype=torch.int32, device="cuda")
    rows_buf = [torch.zeros(K, dtype=torch.int32, device="cuda") for _ in range(2)]
    cnt_buf = [torch.zeros(1, dtype=torch.int32, device="cuda") for _ in range(2)]
    o = Outs(n1, n2, r)
    Ah = torch.zeros(n1, r, dtype=torch.complex64, device="cuda")
    rows_h = np.arange(n1, dtype=np.int32)
    worst, fp64_agree = {}, 0
    for t in range(Tn):
        nxt = dict(K_next=K, rows_next=rows_buf[(t + 1) % 2], n_next=cnt_buf[(t + 1) % 2])
        if t < warm:
            fr = seq.frame(rows=full, y=Kd[t], y_full=True, **o.kw(), **nxt)
        else:
            fr = seq.frame(rows=rows_buf[t % 2], n_rows_dev=cnt_buf[t % 2], y=Kd[t], y_full=True, **o.kw(), **nxt)
        seq.push(fr)
        s = ora.push_lines(rows_h, c["kspace"][t][rows_h])
        e = compare_step(o, s, f"t={t + 1}")
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0), v)
        seq.factors(Ahat=Ah)
        nr_ = int(host(cnt_buf[(t + 1) % 2])[0])
        g_rows = host(rows_buf[(t + 1) % 2])[:nr_].copy()
        o_rows, _ = oracle.draw_lines(host(Ah), n2, K, 77, 3, t + 2)
        assert np.array_equal(o_rows, g_rows), f"row draw differs at t={t + 2}"
        own, _ = oracle.draw_lines(ora.kspace_factors()[0], n2, K, 77, 3, t + 2)
        fp64_agree += int(np.array_equal(own, g_rows))
        rows_h = g_rows if t + 1 >= warm else np.arange(n1, dtype=np.int32)
    print("config 3 worst NRMSE", worst, f"oracle's own FP64 draws agree {fp64_agree}/{Tn}", flush=True)
    assert seq.status() == 0
    seq.close()


def test_step_many_with_draws_equals_push_frame(T):
    print("step_many with draws", flush=True)
    specs = [(128, 128, 16), (256, 256, 32), (128, 128, 8), (192, 160, 24)]
    rng = np.random.default_rng(5)
    A_seqs, B_seqs, data = [], [], []
    for k, (n1, n2, r) in enumerate(specs):
        _, A0, B0 = _random_state(n1, n2, r, 900 + k)
        A_seqs.append(T.Sequence(n1, n2, r, 0.05, dev(A0), dev(B0), seed=5, stream_id=k))
        B_seqs.append(T.Sequence(n1, n2, r, 0.05, dev(A0), dev(B0), seed=5, stream_id=k))
        data.append(dev(cn(rng, (6, n1, n2), 1e-3).astype(np.complex64)))
    bufs = {}
    for side in ("batch", "solo"):
        bufs[side] = [dict(rows=[torch.zeros(n1 // 8, dtype=torch.int32, device="cuda") for _ in range(2)],
                           cnt=[torch.zeros(1, dtype=torch.int32, device="cuda") for _ in range(2)],
                           out=Outs(n1, n2, r)) for (n1, n2, r) in specs]
    for t in range(6):
        frames = []
        for k, (n1, n2, r) in enumerate(specs):
            for side, sq in (("batch", A_seqs[k]), ("solo", B_seqs[k])):
                b = bufs[side][k]
                nxt = dict(K_next=n1 // 8, rows_next=b["rows"][(t + 1) % 2], n_next=b["cnt"][(t + 1) % 2])
                if t == 0:
                    fr = sq.frame(rows=torch.arange(n1, dtype=torch.int32, device="cuda"), y=data[k][t],
                                  y_full=True, **b["out"].kw(), **nxt)
                else:
                    fr = sq.frame(rows=b["rows"][t % 2], n_rows_dev=b["cnt"][t % 2], y=data[k][t], y_full=True,
                                  **b["out"].kw(), **nxt)
                if side == "batch":
                    frames.append(fr)
                else:
                    sq.push(fr)
        T.step_many(A_seqs, frames)
        for k in range(len(specs)):
            bb, bs = bufs["batch"][k], bufs["solo"][k]
            assert np.array_equal(host(bb["out"].X), host(bs["out"].X))
            assert np.array_equal(host(bb["cnt"][(t + 1) % 2]), host(bs["cnt"][(t + 1) % 2]))
            n_ = int(host(bb["cnt"][(t + 1) % 2])[0])
            assert np.array_equal(host(bb["rows"][(t + 1) % 2])[:n_], host(bs["rows"][(t + 1) % 2])[:n_])
    for s in A_seqs + B_seqs:
        assert s.status() == 0
        s.close()


@pytest.mark.parametrize("graph", [False, True])
def test_prepared_batch_replays_equal_step_many(T, graph):
    """Prepared batches (descriptors fixed at creation; launched directly or
    replayed from a graph) run in a cycle give bit-identical outputs and draws
    to tsl_step_many on twin sequences; closing a sequence invalidates the
    batches that hold it."""
    print(f"prepared batch replays, graph={graph}", flush=True)
    specs = [(128, 128, 16, "kspace"), (256, 256, 32, "kspace"), (128, 128, 8, "frame"),
             (192, 160, 24, "kspace")]
    rng = np.random.default_rng(11)
    P_seqs, M_seqs, data = [], [], []
    for k, (n1, n2, r, route) in enumerate(specs):
        _, A0, B0 = _random_state(n1, n2, r, 950 + k)
        P_seqs.append(T.Sequence(n1, n2, r, 0.05, dev(A0), dev(B0), seed=7, stream_id=k, route=route))
        M_seqs.append(T.Sequence(n1, n2, r, 0.05, dev(A0), dev(B0), seed=7, stream_id=k, route=route))
        data.append(dev(cn(rng, (3, n1, n2), 1e-3).astype(np.complex64)))
    bufs = {}
    for side in ("prep", "many"):
        bufs[side] = [dict(rows=[torch.zeros(n1 // 8, dtype=torch.int32, device="cuda") for _ in range(2)],
                           cnt=[torch.zeros(1, dtype=torch.int32, device="cuda") for _ in range(2)],
                           out=Outs(n1, n2, r)) for (n1, n2, r, _) in specs]
    full = {n1: torch.arange(n1, dtype=torch.int32, device="cuda") for (n1, _, _, _) in specs}

    def frames_for(side, seqs, t):
        fr = []
        for k, (n1, n2, r, _) in enumerate(specs):
            b = bufs[side][k]
            nxt = dict(K_next=n1 // 8, rows_next=b["rows"][(t + 1) % 2], n_next=b["cnt"][(t + 1) % 2])
            y = data[k][t % 3]
            if t == 0:
                fr.append(seqs[k].frame(rows=full[n1], y=y, y_full=True, **b["out"].kw(), **nxt))
            else:
                fr.append(seqs[k].frame(rows=b["rows"][t % 2], n_rows_dev=b["cnt"][t % 2], y=y, y_full=True,
                                        **b["out"].kw(), **nxt))
        return fr

    # step 0 (all rows), then a cycle of 6 steps (row-buffer parity x data frame)
    prepared = {key: T.PreparedStep(P_seqs, frames_for("prep", P_seqs, key), graph=graph) for key in range(7)}
    for t in range(14):
        key = t if t < 7 else 1 + (t - 1) % 6
        prepared[key].launch()
        T.step_many(M_seqs, frames_for("many", M_seqs, key))
        for k in range(len(specs)):
            bp, bm = bufs["prep"][k], bufs["many"][k]
            for name in ("X", "A", "B", "g"):
                assert np.array_equal(host(getattr(bp["out"], name)), host(getattr(bm["out"], name))), (t, k, name)
            cp, cm = host(bp["cnt"][(t + 1) % 2]), host(bm["cnt"][(t + 1) % 2])
            assert np.array_equal(cp, cm), (t, k)
            n_ = int(cp[0])
            assert np.array_equal(host(bp["rows"][(t + 1) % 2])[:n_], host(bm["rows"][(t + 1) % 2])[:n_])
    for s in P_seqs + M_seqs:
        assert s.status() == 0
    P_seqs[2].close()
    with pytest.raises(T.TslError) as ei:
        prepared[3].launch()
    assert ei.value.code == T.EINVAL
    for p in prepared.values():
        p.close()
        p.close()
    for s in P_seqs[:2] + P_seqs[3:] + M_seqs:
        s.close()


def test_device_row_count_out_of_range_latches(T):
    n1, n2, r = 64, 64, 4
    _, A0, B0 = _random_state(n1, n2, r, 8)
    seq = T.Sequence(n1, n2, r, 0.1, dev(A0), dev(B0))
    rows = torch.arange(8, dtype=torch.int32, device="cuda")
    cnt = torch.tensor([65], dtype=torch.int32, device="cuda")
    y = torch.zeros(n1, n2, dtype=torch.complex64, device="cuda")
    seq.push(seq.frame(rows=rows, n_rows_dev=cnt, y=y, y_full=True))
    assert seq.status(clear=True) == T.EINVAL
    seq.close()


@pytest.mark.parametrize("n1,n2,r,nrows,kind", [(256, 256, 32, 32, "lines"), (128, 128, 64, 40, "lines"),
                                                (64, 64, 8, 0, "points"), (120, 200, 5, 37, "lines")])
def test_frame_info_matches_oracle(T, n1, n2, r, nrows, kind):
    """info_out carries alpha_t, alpha_bar_t, mu_t and the pivot ratio of the
    ridge Gram; each matches the oracle's to 1e-4 relative on every frame (both
    sides in FP64, from factors that agree to the parity bar)."""
    print(f"frame info {kind} {n1}x{n2} r={r}", flush=True)
    rng, A0, B0 = _random_state(n1, n2, r, 4 * n1 + n2 + r)
    ora = oracle.TslOracle(n1, n2, r, 0.05, A0, B0)
    seq = T.Sequence(n1, n2, r, 0.05, dev(A0), dev(B0))
    info = torch.zeros(4, dtype=torch.float64, device="cuda")
    worst = 0.0
    for t in range(4):
        if kind == "lines":
            rows = np.sort(rng.choice(n1, nrows, replace=False)).astype(np.int32)
            Y = cn(rng, (nrows, n2), 50.0 / (n1 * n2)).astype(np.complex64)
            s = ora.push_lines(rows, Y)
            fr = seq.frame(rows=dev(rows), y=dev(Y), info_out=info)
        else:
            mask = rng.random((n1, n2)) < 0.25
            Y = cn(rng, (n1, n2), 50.0 / (n1 * n2)).astype(np.complex64)
            s = ora.push_points(mask, Y)
            fr = seq.frame(mask=dev(mask.astype(np.uint8)), y=dev(Y), info_out=info)
        seq.push(fr)
        got = host(info)
        want = np.array([s.alpha, s.alpha_bar, s.mu, s.pivot_ratio])
        rel = np.abs(got - want) / np.abs(want)
        worst = max(worst, float(rel.max()))
        assert np.all(rel <= TOL), f"t={t + 1}: got {got}, want {want}"
    print(f"frame info worst relative error {worst:.2e}, last pivot ratio {got[3]:.3e}", flush=True)
    assert seq.status() == 0
    seq.close()


# ---------------------------------------------------------------------------- point sampling (eq. 13)
@pytest.mark.parametrize("n1,n2,r,K", [(64, 64, 8, 1024), (120, 200, 5, 500), (256, 256, 32, 8192),
                                       (512, 64, 128, 300), (8, 16, 3, 40)])
def test_point_sampler_bit_exact_on_device_factors(T, n1, n2, r, K):
    """tsl_sample_points draws from the device's F_l A and F_r B exactly what
    the oracle's point sampler draws from the same (exported) factors."""
    print(f"point sampler {n1}x{n2} r={r} K={K}", flush=True)
    rng, A0, B0 = _random_state(n1, n2, r, 3 * n1 + n2 + r)
    seq = T.Sequence(n1, n2, r, 0.05, dev(A0), dev(B0), seed=2024, stream_id=r)
    for _ in range(2):
        mask = rng.random((n1, n2)) < 0.3
        seq.push_points(dev(mask.astype(np.uint8)), dev(cn(rng, (n1, n2), 50.0 / (n1 * n2)).astype(np.complex64)))
    m = torch.zeros(n1, n2, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    dr = torch.zeros(K, dtype=torch.int32, device="cuda")
    seq.sample_points(K, m, cnt, draws_out=dr)
    Ah = torch.zeros(n1, r, dtype=torch.complex64, device="cuda")
    Bh = torch.zeros(n2, r, dtype=torch.complex64, device="cuda")
    seq.factors(Ahat=Ah, Bhat=Bh)
    want_mask, want_draws = oracle.draw_points(host(Ah), host(Bh), K, 2024, r, 3)
    assert np.array_equal(host(dr), want_draws[:, 0] * n2 + want_draws[:, 1])
    assert np.array_equal(host(m).astype(bool), want_mask)
    assert int(host(cnt)[0]) == int(want_mask.sum())
    assert seq.status() == 0
    seq.close()


def test_point_sampled_trajectory_matches_oracle(T):
    """Six frames of the 64 x 64, R = 8 low-rank sequence, each acquired at the
    entries the device drew from the previous frame's factors (the first frame
    at a uniform 25 % mask): masks equal the oracle's draw bit for bit and the
    outputs meet the parity bar."""
    c = I.config1(T=6)
    n, r, K = 64, 8, 1024
    ora = oracle.TslOracle(n, n, r, 0.1, c["A0"], c["B0"])
    seq = T.Sequence(n, n, r, 0.1, dev(c["A0"]), dev(c["B0"]), seed=5, stream_id=9)
    o = Outs(n, n, r)
    m = torch.zeros(n, n, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    Ah = torch.zeros(n, r, dtype=torch.complex64, device="cuda")
    Bh = torch.zeros(n, r, dtype=torch.complex64, device="cuda")
    mask = c["frames"][0].mask
    for t, fr in enumerate(c["frames"]):
        full = np.fft.fft2(fr.truth, norm="ortho").astype(np.complex64)      # the frame's k-space
        s = ora.push_points(mask, full)
        seq.push_points(dev(mask.astype(np.uint8)), dev(full), **o.kw())
        compare_step(o, s, f"t={t + 1}")
        seq.sample_points(K, m, cnt)
        seq.factors(Ahat=Ah, Bhat=Bh)
        want, _ = oracle.draw_points(host(Ah), host(Bh), K, 5, 9, t + 2)
        got = host(m).astype(bool)
        assert np.array_equal(got, want) and int(host(cnt)[0]) == int(want.sum())
        mask = got
    assert seq.status() == 0
    seq.close()
