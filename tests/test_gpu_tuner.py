"""The output-synthesis tile tuner: every tile gives the same frames bit for
bit, and prepared-batch creation records a measured choice (and appends it to
the TSL_TUNE_CACHE file)."""

import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_04104_amd import tsl
    tsl.lib()
    return tsl


def _seqs(T, specs, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k, (n1, n2, r) in enumerate(specs):
        A0 = ((rng.normal(size=(n1, r)) + 1j * rng.normal(size=(n1, r))) / np.sqrt(2 * n1)).astype(np.complex64)
        B0 = ((rng.normal(size=(n2, r)) + 1j * rng.normal(size=(n2, r))) / np.sqrt(2 * n2)).astype(np.complex64)
        out.append(T.Sequence(n1, n2, r, 0.05, torch.from_numpy(A0).cuda(), torch.from_numpy(B0).cuda(),
                              seed=3, stream_id=k))
    return out


def test_every_output_tile_gives_the_same_frames(T):
    specs = [(256, 256, 32)] * 6 + [(160, 192, 48)] * 3 + [(96, 80, 8)] * 2
    rng = np.random.default_rng(4)
    ys = [torch.from_numpy(((rng.normal(size=(n1, n2)) + 1j * rng.normal(size=(n1, n2))) * 0.01)
                           .astype(np.complex64)).cuda() for (n1, n2, _) in specs]
    results = []
    for tile in ("128x64", "64x64", "128x128"):
        print(f"output tile {tile}", flush=True)
        for (n1, n2, r) in set(specs):
            T.set_output_tile(n1, n2, r, specs.count((n1, n2, r)), tile)
        T.set_output_tile(256, 256, 32, 6, tile)
        T.set_output_tile(160, 192, 48, 3, tile)
        T.set_output_tile(96, 80, 8, 2, tile)
        seqs = _seqs(T, specs, 9)
        X = [torch.zeros(n1, n2, dtype=torch.complex64, device="cuda") for (n1, n2, _) in specs]
        rows = [torch.arange(n1, dtype=torch.int32, device="cuda") for (n1, _, _) in specs]
        for _ in range(2):
            fr = [q.frame(rows=rw, y=y, y_full=True, X_out=x) for q, rw, y, x in zip(seqs, rows, ys, X)]
            T.step_many(seqs, fr)
        torch.cuda.synchronize()
        results.append([x.cpu().numpy() for x in X])
        for q in seqs:
            assert q.status() == 0
            q.close()
    for other in results[1:]:
        for a, b in zip(results[0], other):
            assert np.array_equal(a, b)


def test_prepared_batch_creation_records_a_measured_tile(T, tmp_path):
    path = tmp_path / "tune.txt"
    os.environ["TSL_TUNE_CACHE"] = str(path)
    try:
        specs = [(192, 192, 16)] * 5              # a launch kind no other test uses
        seqs = _seqs(T, specs, 11)
        X = [torch.zeros(192, 192, dtype=torch.complex64, device="cuda") for _ in specs]
        y = torch.zeros(192, 192, dtype=torch.complex64, device="cuda")
        rows = torch.arange(192, dtype=torch.int32, device="cuda")
        fr = [q.frame(rows=rows, y=y, y_full=True, X_out=x) for q, x in zip(seqs, X)]
        ps = T.PreparedStep(seqs, fr)
        ps.launch()
        ps.close()
        tile = T.output_tile(192, 192, 16, 5)
        lines = path.read_text().split("\n")
        rec = [ln.split() for ln in lines if ln.startswith("192 192 1 8 ")]
        assert rec and T.OUT_TILES[int(rec[-1][4])] == tile
        print(f"tuned output tile for 5 x 192^2, R = 16: {tile}", flush=True)
        for q in seqs:
            assert q.status() == 0
            q.close()
    finally:
        del os.environ["TSL_TUNE_CACHE"]
