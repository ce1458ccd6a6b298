"""The wave primitives every kernel builds on (DPP scans, lane shifts,
lane reads), checked lane by lane against numpy on random inputs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2608_21826_amd")


@pytest.mark.parametrize("seed,lo,hi", [(0, 0, 1000), (1, -(2**20), 2**20), (2, 0, 256),
                                        (3, 0, 2)])
def test_wave_scans(seed, lo, hi):
    print(f"[prim] wave scans seed={seed}", flush=True)
    rng = np.random.default_rng(seed)
    grid, block = 64, 256
    n = grid * block
    x = rng.integers(lo, hi, size=n).astype(np.int32)
    d_in = torch.from_numpy(x).cuda()
    d_out = torch.zeros(4 * n, dtype=torch.int32, device="cuda")
    pkg.probe(8, d_in, d_out, size=n, grid=grid, block=block)
    out = d_out.cpu().numpy().reshape(n, 4)
    w = x.reshape(-1, 64).astype(np.int64)
    incl = np.cumsum(w, axis=1)
    assert np.array_equal(out[:, 0], incl.ravel().astype(np.int32))  # |sums| < 2^27
    umax = np.maximum.accumulate(w.astype(np.uint32), axis=1)
    assert np.array_equal(out[:, 1].astype(np.uint32), umax.ravel())
    below = np.concatenate([np.zeros((w.shape[0], 1), np.int64), w[:, :-1]], axis=1)
    assert np.array_equal(out[:, 2], below.ravel().astype(np.int32))
    assert np.array_equal(out[:, 3], np.repeat(w[:, 63], 64).astype(np.int32))
