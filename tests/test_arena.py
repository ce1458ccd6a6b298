"""The serving engine's memory arena (admission by footprint) as pure host
logic: first-fit offsets, alignment, Full when no block fits, coalescing on
free, peak tracking; checked against a small reference model."""
import numpy as np
import pytest

import paper_2608_21826_amd as pkg


class Model:
    """Reference first-fit allocator over [0, size)."""

    def __init__(self, size, align):
        self.align = align
        self.size = size - size % align
        self.free = [(0, self.size)] if self.size else []
        self.live = {}

    def alloc(self, n):
        need = max(n, 1)
        need = (need + self.align - 1) // self.align * self.align
        for i, (off, ln) in enumerate(self.free):
            if ln >= need:
                if ln > need:
                    self.free[i] = (off + need, ln - need)
                else:
                    self.free.pop(i)
                self.live[off] = need
                return off
        return None

    def release(self, off):
        ln = self.live.pop(off)
        self.free.append((off, ln))
        self.free.sort()
        merged = []
        for o, l in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((o, l))
        self.free = merged


def test_basic():
    a = pkg.Arena(1 << 16, 256)
    x = a.alloc(1)
    y = a.alloc(300)
    assert (x, y) == (0, 256)
    used, peak, largest = a.usage()
    assert used == 256 + 512 and peak == used and largest == (1 << 16) - used
    assert a.alloc(1 << 17) is None
    a.free(x)
    a.free(y)
    assert a.usage()[0] == 0 and a.usage()[2] == 1 << 16
    with pytest.raises(pkg.BQError):
        a.free(12345)
    a.close()


@pytest.mark.parametrize("seed", range(5))
def test_random_against_model(seed):
    rng = np.random.default_rng(seed)
    size, align = 1 << 20, 256
    a = pkg.Arena(size, align)
    m = Model(size, align)
    live = []
    peak = 0
    for step in range(3000):
        if live and rng.random() < 0.45:
            off = live.pop(int(rng.integers(0, len(live))))
            a.free(off)
            m.release(off)
        else:
            n = int(rng.integers(1, 60000))
            got = a.alloc(n)
            exp = m.alloc(n)
            assert got == exp
            if got is not None:
                live.append(got)
        used = sum(m.live.values())
        peak = max(peak, used)
        u, p, lf = a.usage()
        assert u == used and p == peak
        assert lf == max([l for _, l in m.free], default=0)
    a.close()


def test_small_lane_setting_rejects_a_missing_server():
    """Host-side argument check of the reserved-lane setting (no device)."""
    assert pkg.lib().bq_server_set_small_lanes(None, 0) == pkg.BQ_EINVAL
    assert pkg.lib().bq_server_set_small_lanes(None, 1) == pkg.BQ_EINVAL
