"""Pins of the oracle's particle steps: linear charge assignment (Sec. 3.4), leap-frog
push with linear gather (Sec. 3.6, the two difference equations), removal at the walls
(Sec. 2), and the stable sort by cell (Sec. 3.7)."""
import numpy as np
import pytest


# ------------------------------------------------------------------ deposit
@pytest.mark.parametrize("periodic", [0, 1])
def test_deposit_brute_force(oracle_mod, periodic):
    """w[j] = sum_i max(0, 1 - |x_i - j|) (periodic distance when periodic)."""
    rng = np.random.default_rng(10 + periodic)
    n_cells = 37
    x = rng.uniform(0, n_cells, size=3000)
    x[:5] = [0.0, n_cells - 1e-12, 5.0, 5.5, 36.999]
    w = oracle_mod.deposit(periodic, n_cells, x)
    nodes = np.arange(n_cells if periodic else n_cells + 1)
    d = np.abs(x[:, None] - nodes[None, :])
    if periodic:
        d = np.minimum(d, n_cells - d)
    ref = np.maximum(0.0, 1.0 - d).sum(axis=0)
    assert np.allclose(w, ref, rtol=0, atol=1e-10)
    assert w.sum() == pytest.approx(x.size, rel=1e-14)


def test_deposit_large_brute_force(oracle_mod):
    rng = np.random.default_rng(11)
    n_cells = 256
    x = rng.uniform(0, n_cells, size=10000)
    w = oracle_mod.deposit(0, n_cells, x)
    ref = np.zeros(n_cells + 1)
    for xi in x:  # hat function evaluated node by node
        for j in range(n_cells + 1):
            ref[j] += max(0.0, 1.0 - abs(xi - j))
    assert np.max(np.abs(w - ref)) < 1e-11


# ------------------------------------------------------------------ push
def test_push_zero_field_free_streaming(oracle_mod):
    """E = 0: x_n = x_0 + n v exactly (periodic wrap), v unchanged."""
    n_cells = 64
    rng = np.random.default_rng(1)
    x0 = rng.uniform(0, n_cells, 500)
    v = rng.normal(0, 0.37, 500)
    ef = np.zeros(n_cells)
    x, vx = x0.copy(), v.copy()
    for step in range(1, 41):
        x, vx, fl = oracle_mod.push(1, n_cells, -0.01, ef, x, vx)
        assert np.all(fl == 0)
        assert np.array_equal(vx, v)
    ref = np.mod(x0 + 40 * v, n_cells)
    dist = np.abs(x - ref)
    dist = np.minimum(dist, n_cells - dist)
    assert dist.max() < 1e-11


def test_push_constant_field_closed_form(oracle_mod):
    """Uniform E: v_{n+1/2} = v_{-1/2} + (n+1) kappa E and
    x_{n+1} = x_0 + (n+1) v_{-1/2} + kappa E (n+1)(n+2)/2."""
    n_cells = 4096
    kap, e0 = -2.5e-4, 0.8
    ef = np.full(n_cells + 1, e0)
    x0 = np.array([1000.25, 2000.5, 3000.75])
    vm = np.array([0.1, -0.3, 0.05])
    x, vx = x0.copy(), vm.copy()
    nst = 50
    for _ in range(nst):
        x, vx, fl = oracle_mod.push(0, n_cells, kap, ef, x, vx)
        assert np.all(fl == 0)
    a = kap * e0
    assert np.allclose(vx, vm + nst * a, rtol=0, atol=1e-14)
    assert np.allclose(x, x0 + nst * vm + a * nst * (nst + 1) / 2, rtol=0, atol=1e-11)


def test_push_gather_is_linear_interpolation(oracle_mod):
    n_cells = 10
    ef = np.arange(n_cells + 1, dtype=float) ** 2
    x = np.array([2.25, 7.5, 0.0, 9.999])
    x2, vx, fl = oracle_mod.push(0, n_cells, 1.0, ef, x, np.zeros(4))
    c = np.floor(x)
    f = x - c
    ref = (1 - f) * ef[c.astype(int)] + f * ef[c.astype(int) + 1]
    assert np.allclose(vx, ref, rtol=1e-15)


def test_push_walls(oracle_mod):
    """Bounded: a particle is kept iff 0 <= x < N after the move; it leaves at the side it
    crossed (flag 1 left, 2 right); x = N exactly is outside."""
    n_cells = 16
    ef = np.zeros(n_cells + 1)
    x = np.array([0.5, 15.5, 15.5, 0.5, 3.0, 8.0])
    v = np.array([-0.6, 0.6, 0.5, -0.5, 0.0, -8.0])
    _, _, fl = oracle_mod.push(0, n_cells, 0.0, ef, x, v)
    assert list(fl) == [1, 2, 2, 0, 0, 0]


def test_push_fp32_offset_layout(oracle_mod):
    """FP32 cell + offset: after any push the offset stays in [0, 1), the cell is the
    floor of the FP64 position, and the position agrees with the FP64 update to FP32
    rounding of the offset and velocity."""
    n_cells = 8192
    rng = np.random.default_rng(5)
    m = 20000
    cell = rng.integers(0, n_cells, m)
    off = rng.uniform(0, 1, m).astype(np.float32)
    x0 = cell + off.astype(np.float64)
    v0 = rng.normal(0, 3.0, m).astype(np.float32).astype(np.float64)
    ef = rng.normal(0, 50, n_cells).astype(np.float64)
    x, vx, fl = oracle_mod.push(1, n_cells, -1e-4, ef, x0, v0, fp32_offset=True)
    xd, vxd, _ = oracle_mod.push(1, n_cells, -1e-4, ef, x0, v0, fp32_offset=False)
    c = np.floor(x)
    f = x - c
    assert np.all((f >= 0) & (f < 1))
    assert np.all(f == f.astype(np.float32).astype(np.float64))
    assert np.all(vx == vx.astype(np.float32).astype(np.float64))
    d = np.abs(x - xd)
    d = np.minimum(d, n_cells - d)
    assert d.max() < 4e-6  # a few FP32 ulps of |v| + 1
    assert np.allclose(vx, vxd, rtol=1e-6, atol=1e-7)
    # tiny negative moves that round the offset to 1.0f land at offset 0 of the next cell
    x1, _, _ = oracle_mod.push(1, n_cells, 0.0, np.zeros(n_cells), np.array([10.0]),
                               np.array([-1e-10]), fp32_offset=True)
    assert x1[0] == 10.0


# ------------------------------------------------------------------ sort
@pytest.mark.parametrize("n,n_cells", [(0, 4), (1, 4), (1000, 7), (5000, 300)])
def test_stable_sort_by_cell(oracle_mod, n, n_cells):
    rng = np.random.default_rng(n)
    cells = rng.integers(0, n_cells, n).astype(np.int32)
    perm = oracle_mod.stable_sort_by_cell(cells, n_cells)
    assert list(perm) == sorted(range(n), key=lambda i: (cells[i], i))
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert np.array_equal(np.bincount(cells[perm], minlength=n_cells),
                          np.bincount(cells, minlength=n_cells))


def test_stable_sort_all_same_cell(oracle_mod):
    cells = np.full(100, 3, dtype=np.int32)
    assert np.array_equal(oracle_mod.stable_sort_by_cell(cells, 5), np.arange(100))
