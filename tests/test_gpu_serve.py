"""Batched and served steps give each scan the result it gets alone.

A scan's frames are processed the same way whether its step runs alone
(tsl_push_frame) or inside a batch with other scans of other shapes and ranks
(tsl_step_many under the continuous-batching server).  Scans whose group shares
its rank bucket run the same code path as alone, so their results, including the
rows drawn on the device, must be identical to the bit; mixing rank buckets in
one shape group changes only summation orders inside the R x R work, so those
results must agree within 1e-5 relative NRMSE.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_04104_amd import tsl
    tsl.lib()
    return tsl


def nr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _scans(SV, I, dev, specs, T_frames, fps, banks, ids):
    out = []
    for k, (n, r) in zip(ids, specs):
        A0, B0 = I.init_factors(n, n, r, I.rng_for(7, k, 3))
        out.append(SV.Scan(k, n, r, 0.05, torch.from_numpy(A0).to(dev), torch.from_numpy(B0).to(dev),
                           banks[n], T_frames, 0.0, fps, t_warm=3))
    return out


def _finals(T, SV, I, dev, specs, banks, plain, ids, T_frames=10):
    got = {}

    def grab(sc):
        A = torch.empty(sc.n, sc.r, dtype=torch.complex64, device=dev)
        B = torch.empty(sc.n, sc.r, dtype=torch.complex64, device=dev)
        sc.seq.factors(A=A, B=B)
        torch.cuda.synchronize()
        got[sc.sid] = (A.cpu().numpy(), B.cpu().numpy(), sc.X.cpu().numpy(),
                       sc.rows[sc.T % 2].cpu().numpy().copy(), int(sc.cnt[sc.T % 2].item()))

    scans = _scans(SV, I, dev, specs, T_frames, 1e6, banks, ids)
    r = SV.serve(scans, 1 << 34, plain=plain, on_finish=grab)
    assert r["frames"] == len(specs) * T_frames
    return got, r


def test_served_batch_equals_alone_bitwise(T):
    from paper_1609_04104_amd import inputs as I
    from paper_1609_04104_amd import serve as SV
    dev = torch.device("cuda:0")
    print("serve: batched vs alone, same rank buckets", flush=True)
    banks = {n: torch.from_numpy(I.phantom_bank(n, 6, seq=k, config=7)).to(dev) for k, n in enumerate((64, 96))}
    specs = [(64, 12), (64, 16), (96, 9), (96, 14)]          # two shapes, one rank bucket (9..16) each
    mixed, rb = _finals(T, SV, I, dev, specs, banks, plain=False, ids=range(len(specs)))
    assert rb["mean_batch"] > 1.5
    for k, spec in enumerate(specs):
        alone, _ = _finals(T, SV, I, dev, [spec], {spec[0]: banks[spec[0]]}, plain=True, ids=[k])
        a, m = alone[k], mixed[k]
        for x, y in zip(a[:3], m[:3]):
            assert np.array_equal(x, y), f"scan {k} differs from its run alone"
        assert a[4] == m[4] and np.array_equal(a[3][:a[4]], m[3][:m[4]])


def test_mixed_rank_group_matches_alone(T):
    from paper_1609_04104_amd import inputs as I
    print("step_many: ranks 6 / 40 / 20 in one shape group vs alone", flush=True)
    dev = torch.device("cuda:0")
    n, frames = 96, 6
    bank = I.phantom_bank(n, frames, seq=3, config=7)
    ranks = [6, 40, 20]
    rng = np.random.default_rng(5)
    rowsets = [np.sort(rng.choice(n, 24, replace=False)).astype(np.int32) for _ in range(frames)]
    inits = [I.init_factors(n, n, r, I.rng_for(7, 10 + k, 3)) for k, r in enumerate(ranks)]

    def run(batched):
        seqs = [T.Sequence(n, n, r, 0.05, torch.from_numpy(A0).to(dev), torch.from_numpy(B0).to(dev))
                for r, (A0, B0) in zip(ranks, inits)]
        X = [torch.empty(n, n, dtype=torch.complex64, device=dev) for _ in seqs]
        for t in range(frames):
            rows = torch.from_numpy(rowsets[t]).to(dev)
            y = torch.from_numpy(np.ascontiguousarray(bank[t][rowsets[t]])).to(dev)
            fr = [q.frame(rows=rows, y=y, X_out=X[k]) for k, q in enumerate(seqs)]
            if batched:
                T.step_many(seqs, fr)
            else:
                for q, f in zip(seqs, fr):
                    q.push(f)
        torch.cuda.synchronize()
        out = []
        for k, q in enumerate(seqs):
            A = torch.empty(n, ranks[k], dtype=torch.complex64, device=dev)
            q.factors(A=A)
            torch.cuda.synchronize()
            out.append((A.cpu().numpy(), X[k].cpu().numpy()))
            assert q.status() == 0
            q.close()
        return out

    alone, mixed = run(False), run(True)
    for k in range(len(ranks)):
        assert nr(mixed[k][0], alone[k][0]) < 1e-5
        assert nr(mixed[k][1], alone[k][1]) < 1e-5
