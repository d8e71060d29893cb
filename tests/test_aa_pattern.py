"""CPU model of the in-place A-A access pattern of the step kernel.

The model below restates, in integer index arithmetic, the load and store
rules the HIP step kernel uses (own slots in even steps; upstream slot opp(i)
on load and downstream slot i on store in odd steps; half-way bounce-back,
isothermal anti-bounce-back and the adiabatic same-direction copy through the
side buffer).  It checks, without a GPU:
  * every address stays inside its buffer;
  * no slot is written twice in one step, and in odd steps the only slots a
    thread writes that it did not read are those no thread reads (so the
    in-place update is race-free);
  * a sequence of steps with an arbitrary per-node "collision" reproduces
    plain two-array pull streaming with the wall rules of Eqs 34-36 exactly.
"""
import numpy as np
import pytest

EX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
EY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
W = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4


def d5slot(i):
    return 0 if i in (2, 4) else (1 if i in (5, 8) else 2)


class Model:
    def __init__(self, nx, ny):
        self.nx, self.ny = nx, ny
        self.px = (nx + 63) // 64 * 64
        self.plane = self.px * ny
        self.pop = np.full(27 * self.plane, np.nan)
        self.d5 = np.full(6 * self.px, np.nan)
        self.reads, self.writes = [], []

    def _rd(self, a):
        assert 0 <= a < self.pop.size
        self.reads.append(a)
        return self.pop[a]

    def _wr(self, a, v):
        assert 0 <= a < self.pop.size
        self.writes.append(a)
        self.pop[a] = v

    def _d5rd(self, a):
        assert 0 <= a < self.d5.size
        return self.d5[a]

    def _d5wr(self, a, v):
        assert 0 <= a < self.d5.size
        self.d5[a] = v

    def load(self, x, y, odd, log=True):
        nx, ny, px, pl = self.nx, self.ny, self.px, self.plane
        rd = self._rd if log else (lambda a: self.pop[a])
        n = y * px + x
        xl, xr, yb, yt = x == 0, x == nx - 1, y == 0, y == ny - 1
        v = np.zeros((3, 9))
        for i in range(9):
            if not odd:
                for l in range(3):
                    v[l, i] = rd(pl * (9 * l + i) + n)
                continue
            outx = (EX[i] == 1 and xl) or (EX[i] == -1 and xr)
            outy = (EY[i] == 1 and yb) or (EY[i] == -1 and yt)
            out = outx or outy
            a = pl * i + n if out else pl * OPP[i] + n - EX[i] - EY[i] * px
            v[0, i] = rd(a)
            v[1, i] = rd(pl * 9 + a)
            if i == 0:
                v[2, i] = rd(pl * 18 + a)
            elif outy:
                v[2, i] = self._d5rd(((0 if EY[i] == 1 else 3) + d5slot(i)) * px + x)
            else:
                t = rd(pl * 18 + a)
                v[2, i] = ((W[i] if xl else -W[i]) - t) if outx else t
        return v

    def store(self, x, y, odd, v):
        nx, ny, px, pl = self.nx, self.ny, self.px, self.plane
        n = y * px + x
        xl, xr, yb, yt = x == 0, x == nx - 1, y == 0, y == ny - 1
        for i in range(9):
            if not odd:
                for l in range(3):
                    self._wr(pl * (9 * l + OPP[i]) + n, v[l, i])
                continue
            outx = (EX[i] == 1 and xr) or (EX[i] == -1 and xl)
            outy = (EY[i] == 1 and yt) or (EY[i] == -1 and yb)
            out = outx or outy
            a = pl * OPP[i] + n if out else pl * i + n + EX[i] + EY[i] * px
            self._wr(a, v[0, i])
            self._wr(pl * 9 + a, v[1, i])
            if i == 0:
                self._wr(pl * 18 + a, v[2, i])
            elif not out:
                self._wr(pl * 18 + a, v[2, i])
                if (EY[i] == 1 and yb) or (EY[i] == -1 and yt):
                    self._wr(pl * (18 + i) + n + EX[i], v[2, i])
            elif not outy:
                t = (W[i] if EX[i] == -1 else -W[i]) - v[2, i]
                self._wr(pl * 18 + a, t)
                if EY[OPP[i]] == 1 and y == 1:
                    self._wr(pl * 18 + a - px, t)
                if EY[OPP[i]] == -1 and y == ny - 2:
                    self._wr(pl * 18 + a + px, t)
        if not odd:
            g = v[2]
            if yb:
                self._d5wr(0 * px + x, g[2])
                if not xr:
                    self._d5wr(1 * px + x + 1, g[5])
                if not xl:
                    self._d5wr(2 * px + x - 1, g[6])
            if y == 1:
                if xl:
                    self._d5wr(1 * px + 0, W[5] - g[7])
                if xr:
                    self._d5wr(2 * px + nx - 1, -W[6] - g[8])
            if yt:
                self._d5wr(3 * px + x, g[4])
                if not xr:
                    self._d5wr(4 * px + x + 1, g[8])
                if not xl:
                    self._d5wr(5 * px + x - 1, g[7])
            if y == ny - 2:
                if xl:
                    self._d5wr(4 * px + 0, W[8] - g[6])
                if xr:
                    self._d5wr(5 * px + nx - 1, -W[7] - g[5])


def ab_stream(post):
    """Two-array pull streaming with the cavity walls (Eqs 34-36): post has
    shape (3, 9, ny, nx); returns the populations after streaming."""
    _, _, ny, nx = post.shape
    out = np.full_like(post, np.nan)
    for y in range(ny):
        for x in range(nx):
            for i in range(9):
                sx, sy = x - EX[i], y - EY[i]
                inx, iny = 0 <= sx < nx, 0 <= sy < ny
                if inx and iny:
                    out[:, i, y, x] = post[:, i, sy, sx]
                else:
                    out[0, i, y, x] = post[0, OPP[i], y, x]
                    out[1, i, y, x] = post[1, OPP[i], y, x]
                    if not inx:
                        thw = 0.5 if sx < 0 else -0.5
                        out[2, i, y, x] = -post[2, OPP[i], y, x] + 2 * W[i] * thw
    for x in range(nx):
        for i in range(9):
            if EY[i] == 1:
                out[2, i, 0, x] = out[2, i, 1, x]
            elif EY[i] == -1:
                out[2, i, ny - 1, x] = out[2, i, ny - 2, x]
    return out


@pytest.mark.parametrize("nx,ny", [(4, 4), (7, 5), (5, 9), (66, 4)])
def test_aa_matches_pull_streaming_and_is_race_free(nx, ny):
    rng = np.random.default_rng(nx * 100 + ny)
    m = Model(nx, ny)
    F = rng.standard_normal((3, 9, ny, nx))
    # initial state in the even layout: own slots hold f_i(x, 0)
    for l in range(3):
        for i in range(9):
            for y in range(ny):
                m.pop[m.plane * (9 * l + i) + y * m.px: m.plane * (9 * l + i) + y * m.px + nx] = F[l, i, y]
    for t in range(6):
        odd = bool(t & 1)
        kick = rng.standard_normal((3, 9, ny, nx))
        m.reads, m.writes = [], []
        per_node_reads, per_node_writes = [], []
        loaded = {}
        for y in range(ny):
            for x in range(nx):
                r0 = len(m.reads)
                loaded[(x, y)] = m.load(x, y, odd)
                per_node_reads.append(set(m.reads[r0:]))
        for y in range(ny):
            for x in range(nx):
                w0 = len(m.writes)
                m.store(x, y, odd, loaded[(x, y)] + kick[:, :, y, x])
                per_node_writes.append(set(m.writes[w0:]))
        # race freedom: no slot written twice; every slot written by another
        # node than its reader is read by nobody in this step
        assert len(m.writes) == len(set(m.writes))
        all_reads = set(m.reads)
        for r, w in zip(per_node_reads, per_node_writes):
            assert r <= w
            assert (w - r).isdisjoint(all_reads)
        # the AB reference: collide (add the same kick), then pull-stream
        ref = ab_stream(F + kick)
        nxt = bool((t + 1) & 1)
        got = np.zeros_like(ref)
        for y in range(ny):
            for x in range(nx):
                got[:, :, y, x] = m.load(x, y, nxt, log=False)
        np.testing.assert_array_equal(got, ref)
        F = ref
