"""Host-side device-memory arena (hoqri_arena_*): first fit, coalescing, errors.

Checked against a plain Python model of the same policy: blocks are 256-byte
granules, a request takes the lowest-addressed free block that is large
enough, and freeing merges a block with free neighbours.
"""
import numpy as np
import pytest

from paper_2510_16930_amd import _lib as H

G = 256


class Model:
    def __init__(self, size):
        self.size = size // G * G
        self.free = {0: self.size}
        self.live = {}

    def alloc(self, n):
        need = max(1, n)
        need = (need + G - 1) // G * G
        for off in sorted(self.free):
            if self.free[off] >= need:
                sz = self.free.pop(off)
                if sz > need:
                    self.free[off + need] = sz - need
                self.live[off] = need
                return off
        return None

    def release(self, off):
        sz = self.live.pop(off)
        if off + sz in self.free:
            sz += self.free.pop(off + sz)
        prev = [o for o in self.free if o + self.free[o] == off]
        if prev:
            off2 = prev[0]
            sz += self.free.pop(off2)
            off = off2
        self.free[off] = sz

    def stats(self):
        return sum(self.live.values()), max(self.free.values(), default=0), len(self.live)


def test_first_fit_and_coalescing_match_model():
    rng = np.random.default_rng(0)
    size = 1 << 20
    a, m = H.Arena(size), Model(size)
    live = []
    for _ in range(3000):
        if live and rng.random() < 0.45:
            off = live.pop(int(rng.integers(len(live))))
            a.free(off)
            m.release(off)
        else:
            n = int(rng.integers(1, 40000))
            o1, o2 = a.alloc(n), m.alloc(n)
            assert o1 == o2
            if o1 is not None:
                assert o1 % G == 0
                live.append(o1)
        assert a.stats() == m.stats()
    for off in live:
        a.free(off)
    assert a.stats() == (0, size, 0)  # everything merged back into one block


def test_full_and_bad_free():
    a = H.Arena(4096)
    offs = [a.alloc(1000) for _ in range(4)]
    assert offs == [0, 1024, 2048, 3072]
    assert a.alloc(1) is None
    with pytest.raises(H.HoqriError):
        a.free(100)           # not the start of a block
    a.free(1024)
    with pytest.raises(H.HoqriError):
        a.free(1024)          # already free
    assert a.alloc(1024) == 1024
    assert a.alloc(2000) is None  # 0 free bytes left


def test_no_blocks_overlap():
    rng = np.random.default_rng(1)
    a = H.Arena(1 << 16)
    live = {}
    for _ in range(2000):
        if live and rng.random() < 0.5:
            off = list(live)[int(rng.integers(len(live)))]
            a.free(off)
            live.pop(off)
        else:
            n = int(rng.integers(1, 3000))
            off = a.alloc(n)
            if off is not None:
                live[off] = n
        spans = sorted((o, o + n) for o, n in live.items())
        for (s0, e0), (s1, e1) in zip(spans, spans[1:]):
            assert e0 <= s1
        assert all(e <= 1 << 16 for _, e in spans)
