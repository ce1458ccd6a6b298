"""sssp_bf_noalloc (the entry point for callers that cannot allocate)
against sssp_bf through the C ABI: two calls in a row on one device, the
second with a smaller input, each bit-exact to sssp_bf with a context and to
the oracle; the size limit is an error, not a fault."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2608_21826_amd")

DEV = torch.device("cuda:0")


def dev_csr(g):
    return (torch.from_numpy(g.offsets).to(DEV), torch.from_numpy(g.cols).to(DEV),
            torch.from_numpy(g.w).to(DEV))


def both(g, launch=None):
    off, col, w = dev_csr(g)
    print(f"[noalloc] {g.name} n={g.n} m={g.m} launch={launch}", flush=True)
    d0 = torch.full((g.n,), -5, dtype=torch.int64, device=DEV)
    p0 = torch.full((g.n,), -5, dtype=torch.int32, device=DEV)
    neg0 = pkg.sssp_bf_noalloc(off, col, w, g.src, d0, p0, launch=launch, validate=True)
    ctx = pkg.SsspContext(g.n, g.m)
    d1, p1, neg1 = ctx.solve(off, col, w, g.src, launch=launch)
    ctx.close()
    torch.cuda.synchronize()
    return (d0.cpu().numpy(), p0.cpu().numpy(), neg0), (d1.cpu().numpy(), p1.cpu().numpy(), neg1)


@pytest.mark.parametrize("launch", [None, {"segments": 1, "ticket_batch": 4},
                                    {"wg_count": 64, "flags": pkg.BQ_F_BWD},
                                    {"bucket_width": 4, "segments": 2}])
def test_noalloc_equals_sssp_bf_twice_then_smaller(launch):
    big = synth.erdos_renyi(200_000, 8, seed=synth.SEED_BASE + 4)   # the served ER graph
    small = synth.potential_random(3000, 24000, seed=4242)
    for g in (big, small):
        (d0, p0, n0), (d1, p1, n1) = both(g, launch)
        assert n0 == n1 is False
        assert np.array_equal(d0, d1) and np.array_equal(p0, p1)
        d_ref, p_ref, neg = oracle.sssp(g, method="fifo")
        assert not neg and np.array_equal(d0, d_ref) and np.array_equal(p0, p_ref)


def test_noalloc_negative_cycle_and_marking():
    g = synth.road(48, plant_cycle=True, seed=7950)
    off, col, w = dev_csr(g)
    d = torch.empty(g.n, dtype=torch.int64, device=DEV)
    p = torch.empty(g.n, dtype=torch.int32, device=DEV)
    assert pkg.sssp_bf_noalloc(off, col, w, g.src, d, p)
    assert pkg.sssp_bf_noalloc(off, col, w, g.src, d, p, neg_inf=True)
    d_ref, p_ref, neg = oracle.neg_inf(g)
    assert neg
    assert np.array_equal(d.cpu().numpy(), d_ref) and np.array_equal(p.cpu().numpy(), p_ref)


def test_noalloc_rejects_inputs_beyond_its_array():
    """RMAT scale 19 needs more than the fixed array with 8 segments:
    BQ_EBUSY before any device work; with one segment it fits and is exact."""
    g = synth.rmat(19, 16, seed=12)
    off, col, w = dev_csr(g)
    d = torch.empty(g.n, dtype=torch.int64, device=DEV)
    p = torch.empty(g.n, dtype=torch.int32, device=DEV)
    with pytest.raises(pkg.BQError) as ei:
        pkg.sssp_bf_noalloc(off, col, w, g.src, d, p, launch={"segments": 8, "wg_count": 64})
    assert ei.value.status == pkg.BQ_EBUSY
    assert not pkg.sssp_bf_noalloc(off, col, w, g.src, d, p, launch={"segments": 1})
    d_ref, p_ref, _ = oracle.sssp(g, method="fifo")
    assert np.array_equal(d.cpu().numpy(), d_ref) and np.array_equal(p.cpu().numpy(), p_ref)
