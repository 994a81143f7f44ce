"""The allocation-free batched step (tsl_step_many_noalloc) against tsl_step_many.

Two identical sets of sequences advance side by side: one through
tsl_step_many, the other through tsl_step_many_noalloc, whose descriptors live
in the library's fixed device array.  Two calls in a row, the second with a
smaller batch (so the array keeps part of the first call's descriptors), then
the first composition again.  Every output (X_t, A[t], B[t], gamma_t) must meet
the parity bar (relative NRMSE <= 1e-4; the kernels are the same, so equality is
expected) and the rows drawn on the device must be equal bit for bit.
"""

import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_04104_amd import tsl
    tsl.lib()
    return tsl


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def nr(a, b):
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def cn(rng, shape, var=1.0):
    return rng.normal(0, np.sqrt(var / 2), shape) + 1j * rng.normal(0, np.sqrt(var / 2), shape)


# (n1, n2, r, kind): kind "k" line mask on the k-space route, "f" line mask on
# the frame route, "p" point mask.  Fourteen frames take two descriptor uploads.
SPECS = [(128, 128, 16, "k"), (256, 256, 32, "k"), (192, 160, 24, "f"), (64, 64, 8, "p"),
         (128, 128, 64, "k"), (256, 256, 32, "f"), (96, 80, 12, "k"), (128, 128, 16, "k"),
         (64, 64, 8, "k"), (160, 192, 48, "k"), (64, 64, 8, "p"), (256, 256, 32, "k"),
         (120, 200, 5, "f"), (128, 128, 32, "k")]


class Side:
    """One set of sequences with its device buffers."""

    def __init__(self, T, rng_seed):
        rng = np.random.default_rng(rng_seed)
        self.seqs, self.buf = [], []
        for k, (n1, n2, r, kind) in enumerate(SPECS):
            st = np.random.default_rng(700 + k)
            A0 = (cn(st, (n1, r)) / np.sqrt(n1)).astype(np.complex64)
            B0 = (cn(st, (n2, r)) / np.sqrt(n2)).astype(np.complex64)
            self.seqs.append(T.Sequence(n1, n2, r, 0.05, torch.from_numpy(A0).cuda(), torch.from_numpy(B0).cuda(),
                                        seed=9, stream_id=k, route="frame" if kind == "f" else "kspace"))
            K = max(1, n1 // 8)
            self.buf.append(dict(
                K=K, rows=[torch.zeros(K, dtype=torch.int32, device="cuda") for _ in range(2)],
                cnt=[torch.zeros(1, dtype=torch.int32, device="cuda") for _ in range(2)],
                X=torch.zeros(n1, n2, dtype=torch.complex64, device="cuda"),
                A=torch.zeros(n1, r, dtype=torch.complex64, device="cuda"),
                B=torch.zeros(n2, r, dtype=torch.complex64, device="cuda"),
                g=torch.zeros(r, dtype=torch.complex64, device="cuda"),
                t=0))
        del rng

    def frame(self, k, data, masks):
        n1, n2, r, kind = SPECS[k]
        b, q = self.buf[k], self.seqs[k]
        t = b["t"]
        outs = dict(X_out=b["X"], A_out=b["A"], B_out=b["B"], gamma_out=b["g"])
        y = data[k][t % data[k].shape[0]]
        if kind == "p":
            return q.frame(mask=masks[k][t % masks[k].shape[0]], y=y, **outs)
        nxt = dict(K_next=b["K"], rows_next=b["rows"][(t + 1) % 2], n_next=b["cnt"][(t + 1) % 2])
        if t == 0:
            return q.frame(rows=torch.arange(n1, dtype=torch.int32, device="cuda"), y=y, y_full=True, **outs, **nxt)
        return q.frame(rows=b["rows"][t % 2], n_rows_dev=b["cnt"][t % 2], y=y, y_full=True, **outs, **nxt)


def _step(T, side, ks, data, masks, fn):
    frames = [side.frame(k, data, masks) for k in ks]
    fn([side.seqs[k] for k in ks], frames)
    for k in ks:
        side.buf[k]["t"] += 1


def _compare(ref, na, ks, tag):
    worst = 0.0
    for k in ks:
        a, b = ref.buf[k], na.buf[k]
        for name in ("X", "A", "B", "g"):
            e = nr(host(b[name]), host(a[name]))
            worst = max(worst, e)
            assert e <= TOL, f"{tag}: sequence {k} {name} NRMSE {e:.3e}"
        if SPECS[k][3] != "p":
            t = a["t"]
            ca, cb = host(a["cnt"][t % 2]), host(b["cnt"][t % 2])
            assert np.array_equal(ca, cb), f"{tag}: sequence {k} row counts differ"
            m = int(ca[0])
            assert np.array_equal(host(a["rows"][t % 2])[:m], host(b["rows"][t % 2])[:m]), \
                f"{tag}: sequence {k} drawn rows differ"
    return worst


def test_noalloc_step_equals_step_many_on_two_calls(T):
    print("tsl_step_many_noalloc vs tsl_step_many: 14 frames, then 3, then 14", flush=True)
    rng = np.random.default_rng(31)
    data = [torch.from_numpy(cn(rng, (3, n1, n2), 1e-3).astype(np.complex64)).cuda() for (n1, n2, _, _) in SPECS]
    masks = [torch.from_numpy((rng.random((3, n1, n2)) < 0.3).astype(np.uint8)).cuda()
             if kind == "p" else None for (n1, n2, _, kind) in SPECS]
    ref, na = Side(T, 1), Side(T, 1)
    everyone = list(range(len(SPECS)))
    few = [3, 8, 12]          # a point mask, a small k-space frame, a frame-route frame
    calls = [everyone, few, everyone]
    worst = 0.0
    for c, ks in enumerate(calls):
        _step(T, ref, ks, data, masks, T.step_many)
        _step(T, na, ks, data, masks, T.step_many_noalloc)
        worst = max(worst, _compare(ref, na, ks, f"call {c + 1} ({len(ks)} frames)"))
        print(f"call {c + 1}: {len(ks)} frames, worst NRMSE {worst:.2e}", flush=True)
    for q in ref.seqs + na.seqs:
        assert q.status() == 0
        q.close()


def test_noalloc_rejects_more_frames_than_its_array(T):
    from paper_1609_04104_amd import tsl
    n1 = n2 = 64
    r = 8
    z = torch.zeros(n1, r, dtype=torch.complex64, device="cuda") + 0.1
    q = T.Sequence(n1, n2, r, 0.05, z, z.clone())
    n = tsl.STATIC_MAX_FRAMES + 1
    hs = (ctypes.c_void_p * n)(*([q.h] * n))
    fs = (tsl.Frame * n)()
    rc = tsl.lib().tsl_step_many_noalloc(hs, n, fs, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == tsl.EINVAL
    assert b"at most" in tsl.lib().tsl_last_error()
    assert q.status() == 0
    q.close()
