"""Pins for the CPU oracle: each test checks the oracle against something other
than itself (closed forms, published generator outputs, symmetries, invariants,
brute force), so that a dropped term, a wrong sign, a wrong index or a
transposed operand in it fails at least one test."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1310_4218_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def tiny(nx=12, ny=10, nz=6, kmin=0, kmax=0, hot=((5, 4, 0, 0),), sigma=3.0, px=3, py=2,
         cc=0.4, cn=0.1, eps=0.01, steps=4, seed=77, alpha=32):
    xs, ys = W.make_splits(nx, ny, px, py)
    return W.Workload(name="tiny", nx=nx, ny=ny, nz=nz, px=px, py=py, xsplit=xs, ysplit=ys,
                      hot=list(hot), sigma=sigma, kmin=kmin, kmax=kmax, steps=steps,
                      c_center=cc, c_nbr=cn, eps=eps, seed=seed, alpha_work=alpha)


# ---------------------------------------------------------------- generator
def test_splitmix64_published_outputs():
    with open(os.path.join(GOLD, "splitmix64.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert rows
    for seed, idx, out in rows:
        assert oracle.splitmix64(int(seed), int(idx)) == int(out)


def test_init_field_distribution():
    q = oracle.init_field(32, 16, 8, seed=5)
    assert q.min() >= -1.0 and q.max() < 1.0
    assert np.all(q * 2 ** 23 == np.round(q * 2 ** 23))          # multiples of 2^-23
    assert abs(q.mean()) < 0.02 and abs(q.var() - 1 / 3) < 0.02  # uniform on [-1, 1)
    # value of cell n is the (n+1)-th generator output, top 24 bits, centred
    n = 1234
    m = oracle.splitmix64(5, n) >> 40
    assert q.reshape(-1)[n] == (m - 2 ** 23) / 2 ** 23


# ---------------------------------------------------------------- stencil (k = 0)
def eigen_field(nx, ny, nz, m, n, l):
    x = np.arange(nx)[None, :, None]
    y = np.arange(ny)[:, None, None]
    z = np.arange(nz)[None, None, :]
    return (np.cos(2 * np.pi * m * x / nx) * np.cos(2 * np.pi * n * y / ny)
            * np.cos(np.pi * l * (z + 0.5) / nz))


@pytest.mark.parametrize("mnl", [(0, 0, 0), (1, 0, 0), (0, 2, 0), (0, 0, 1), (3, 1, 2), (6, 5, 5)])
def test_stencil_eigenmodes(mnl):
    """With no physics the update is linear and shift-invariant: separable cos modes
    (periodic in x, y; DCT-II in z, which meets the mirror ghost exactly) are
    eigenvectors with eigenvalue cc + 2cn[cos(2pi m/nx) + cos(2pi n/ny) + cos(pi l/nz)]."""
    nx, ny, nz = 12, 10, 6
    m, n, l = mnl
    q0 = eigen_field(nx, ny, nz, m, n, l)
    wl = tiny(nx, ny, nz, kmin=0, kmax=0, steps=5)
    q, _, _, _ = oracle.run(wl, q0=q0)
    mu = 0.4 + 0.2 * (math.cos(2 * math.pi * m / nx) + math.cos(2 * math.pi * n / ny)
                      + math.cos(math.pi * l / nz))
    np.testing.assert_allclose(q[0], mu ** 5 * q0, atol=1e-13, rtol=0)


def test_stencil_matches_roll_formulation():
    """Independent formulation of the same update with array rolls (periodic x/y)
    and edge replication (mirror ghost in z)."""
    rng = np.random.default_rng(3)
    q = rng.uniform(-1, 1, size=(7, 9, 5))
    s = oracle.stencil(q, 0.4, 0.1)
    zpad = np.concatenate([q[:, :, :1], q, q[:, :, -1:]], axis=2)
    nb = (np.roll(q, 1, axis=1) + np.roll(q, -1, axis=1) + np.roll(q, 1, axis=0)
          + np.roll(q, -1, axis=0) + zpad[:, :, :-2] + zpad[:, :, 2:])
    np.testing.assert_allclose(s, 0.4 * q + 0.1 * nb, atol=1e-15, rtol=0)


def test_stencil_single_level_centre_weight():
    """nz = 1: both z neighbours are the cell itself (zero flux), so s = 0.6 q + 0.1 (4 lateral)."""
    q = np.zeros((3, 3, 1))
    q[1, 1, 0] = 1.0
    s = oracle.stencil(q, 0.4, 0.1)
    assert s[1, 1, 0] == pytest.approx(0.6, abs=1e-15)
    assert s[0, 1, 0] == pytest.approx(0.1, abs=1e-15)
    assert s[0, 0, 0] == 0.0


def test_mass_conserved_without_physics():
    wl = tiny(16, 12, 7, kmin=0, kmax=0, steps=6)
    q0 = oracle.init_field(16, 12, 7, seed=9)
    m0 = q0.sum()
    _, _, ck, _ = oracle.run(wl, q0=q0)
    np.testing.assert_allclose(ck, m0, atol=1e-12 * np.abs(q0).sum())


@pytest.mark.parametrize("c", [-1.0, -0.5, 0.0, 0.25, 0.7, 1.0])
def test_constant_field_without_physics(c):
    wl = tiny(kmin=0, kmax=0, steps=5)
    q, _, _, _ = oracle.run(wl, q0=np.full((wl.ny, wl.nx, wl.nz), c))
    np.testing.assert_allclose(q, c, atol=4e-15, rtol=0)


@pytest.mark.parametrize("c", [-1.0, 0.0, 1.0])
def test_fixed_points_with_physics(c):
    """-1, 0 and 1 are fixed points of the stencil (weights sum to one) and of
    Phi (q - q^3 = 0), so they survive the full update with physics on."""
    wl = tiny(kmin=1, kmax=40, steps=4)
    q, _, _, _ = oracle.run(wl, q0=np.full((wl.ny, wl.nx, wl.nz), c))
    np.testing.assert_allclose(q, c, atol=1e-14, rtol=0)


# ---------------------------------------------------------------- column map Phi
def test_phi_linear_growth_near_zero():
    """Phi(q) = q + eps(q - q^3) has slope 1 + eps at 0: tiny values grow by (1+eps)^k."""
    q0, k = 1e-12, 50
    s = np.full((1, 1, 1), q0)
    out = oracle.physics(s, np.array([[k]]), eps=0.01)[0, 0, 0]
    assert out == pytest.approx(q0 * 1.01 ** k, rel=1e-12)


def test_phi_contraction_near_one():
    """Slope at +-1 is 1 - 2 eps: a small offset from 1 shrinks by (1 - 2 eps)^k."""
    d, k = 1e-9, 40
    s = np.array([[[1 - d, -1 + d]]])
    out = oracle.physics(s, np.array([[k]]), eps=0.01)[0, 0]
    assert 1 - out[0] == pytest.approx(d * 0.98 ** k, rel=1e-5)
    assert out[1] + 1 == pytest.approx(d * 0.98 ** k, rel=1e-5)


def test_phi_odd_monotone_bounded():
    v = np.linspace(0, 1, 21)
    s = np.concatenate([-v[:0:-1], v]).reshape(1, 1, 41)   # exactly symmetric samples
    out = oracle.physics(s, np.array([[7]]), eps=0.01)[0, 0]
    np.testing.assert_array_equal(out, -out[::-1])          # odd
    assert np.all(np.diff(out) > 0)                          # monotone
    assert np.all(np.abs(out) <= 1.0)
    assert np.all(np.abs(out[1:-1]) >= np.abs(s[0, 0, 1:-1]))  # pushed away from 0


def test_identity_stencil_leaves_only_phi():
    """cc = 1, cn = 0 make the Jacobi step the identity, so the update is Phi^k per cell."""
    wl = tiny(kmin=1, kmax=9, cc=1.0, cn=0.0, steps=1)
    q0 = oracle.init_field(wl.nx, wl.ny, wl.nz, seed=4)[0]
    q, _, _, k = oracle.run(wl, q0=q0)
    ref = oracle.physics(q0, k, eps=0.01)
    np.testing.assert_array_equal(q[0], ref)


# ---------------------------------------------------------------- cost field k
def test_kfield_gaussian_levels():
    """k >= kmin + j exactly where (kmax-kmin) exp(-r^2/(2 sigma^2)) >= j, i.e. where
    r^2 <= 2 sigma^2 ln((kmax-kmin)/j); counted here by brute force over lattice offsets."""
    nx = ny = 64
    sigma, kmin, kmax = 8.0, 1, 32
    k = oracle.kfield(nx, ny, [(32, 32, 0, 0)], 0, sigma, kmin, kmax)
    assert k[32, 32] == kmax and (k == kmax).sum() == 1
    assert k.min() == kmin
    for j in (1, 2, 5, 16, 30, 31):
        bound = 2 * sigma ** 2 * math.log((kmax - kmin) / j)
        count = sum(1 for dx in range(-32, 32) for dy in range(-32, 32)
                    if dx * dx + dy * dy <= bound)
        assert (k >= kmin + j).sum() == count, j


def test_kfield_periodic_minimum_image_and_motion():
    nx, ny = 40, 30
    hot = [(2, 1, 3, -2)]
    k0 = oracle.kfield(nx, ny, hot, 0, 5.0, 1, 50)
    # minimum image: the hotspot at the edge wraps around symmetrically
    assert k0[1, 1] == k0[1, 3] and k0[0, 2] == k0[2, 2]
    assert k0[1, nx - 1] == k0[1, 5] and k0[ny - 1, 2] == k0[3, 2]
    # a moving hotspot translates the field: k_t(x, y) = k_0(x - vx t, y - vy t)
    for t in (1, 7, 45):
        kt = oracle.kfield(nx, ny, hot, t, 5.0, 1, 50)
        np.testing.assert_array_equal(kt, np.roll(np.roll(k0, 3 * t, axis=1), -2 * t, axis=0))


def test_kfield_two_hotspots_is_max():
    nx, ny = 48, 48
    a = oracle.kfield(nx, ny, [(10, 12, 0, 0)], 0, 6.0, 1, 100)
    b = oracle.kfield(nx, ny, [(30, 33, 0, 0)], 0, 6.0, 1, 100)
    ab = oracle.kfield(nx, ny, [(10, 12, 0, 0), (30, 33, 0, 0)], 0, 6.0, 1, 100)
    np.testing.assert_array_equal(ab, np.maximum(a, b))


def test_zero_column_cost_reduces_to_stencil():
    wl = tiny(kmin=0, kmax=0, steps=1)
    q0 = oracle.init_field(wl.nx, wl.ny, wl.nz, seed=3)[0]
    q, _, _, k = oracle.run(wl, q0=q0)
    assert np.all(k == 0)
    np.testing.assert_array_equal(q[0], oracle.stencil(q0))


# ---------------------------------------------------------------- symmetries
def test_odd_symmetry_bit_exact():
    wl = tiny(kmin=1, kmax=30, steps=3)
    q0 = oracle.init_field(wl.nx, wl.ny, wl.nz, seed=8)
    a, _, _, _ = oracle.run(wl, q0=q0)
    b, _, _, _ = oracle.run(wl, q0=-q0)
    np.testing.assert_array_equal(a, -b)


def test_translation_bit_exact():
    """Shifting the initial field and every hotspot by one cell in x shifts the result."""
    wl = tiny(kmin=1, kmax=30, steps=3, hot=((5, 4, 1, 0),))
    q0 = oracle.init_field(wl.nx, wl.ny, wl.nz, seed=8)
    a, _, _, _ = oracle.run(wl, q0=q0)
    b, _, _, _ = oracle.run(wl.replace(hot=[(6, 4, 1, 0)]), q0=np.roll(q0, 1, axis=2))
    np.testing.assert_array_equal(np.roll(a, 1, axis=2), b)


def test_bounded_by_one():
    wl = tiny(kmin=1, kmax=300, steps=6)
    q, _, _, _ = oracle.run(wl)
    assert np.abs(q).max() <= 1.0


# ---------------------------------------------------------------- loads
def test_work_loads():
    wl = tiny(12, 10, 6, kmin=0, kmax=0, steps=1, px=3, py=2, alpha=7)
    _, work, _, _ = oracle.run(wl)
    ncols = [(wl.xsplit[i + 1] - wl.xsplit[i]) * (wl.ysplit[j + 1] - wl.ysplit[j])
             for j in range(wl.py) for i in range(wl.px)]
    np.testing.assert_array_equal(work[0], [7 * 6 * n for n in ncols])
    wl2 = tiny(12, 10, 6, kmin=1, kmax=40, steps=2, px=3, py=2, alpha=7)
    _, work2, _, klast = oracle.run(wl2)
    assert work2[1].sum() == 6 * (7 * 12 * 10 + int(klast.sum()))
    # the chunk layout is row-major over (y-chunk, x-chunk)
    c = 1 * wl2.px + 2
    sub = klast[wl2.ysplit[1]:wl2.ysplit[2], wl2.xsplit[2]:wl2.xsplit[3]]
    assert work2[1][c] == 6 * (7 * sub.size + int(sub.sum()))


def test_dirichlet_splits_valid():
    xs, ys = W.make_splits(2048, 2048, 64, 64, "dirichlet", 20.0, 2005)
    for s, n in ((xs, 2048), (ys, 2048)):
        assert s[0] == 0 and s[-1] == n and len(s) == 65
        d = np.diff(s)
        assert d.min() >= 1
        assert 0.3 < d.min() / 32 and d.max() / 32 < 2.5
    # extreme concentration still yields a valid split
    xs, _ = W.make_splits(40, 40, 40, 2, "dirichlet", 0.05, 1)
    assert np.all(np.diff(xs) == 1)


# ---------------------------------------------------------------- vertical column physics
def test_vertical_constant_columns_fixed():
    """Equal levels give b^3 - q^3 = 0 exactly, so constant columns never change."""
    s = np.zeros((2, 3, 6))
    s[0] = 0.3
    s[1] = -0.7
    out = oracle.physics(s, np.full((2, 3), 25, np.int32), vertical=True)
    np.testing.assert_array_equal(out, s)


def test_vertical_bottom_fixed_and_single_level():
    rng = np.random.default_rng(1)
    s = rng.uniform(-1, 1, size=(3, 4, 7))
    out = oracle.physics(s, np.full((3, 4), 9, np.int32), vertical=True)
    np.testing.assert_array_equal(out[:, :, 0], s[:, :, 0])
    s1 = rng.uniform(-1, 1, size=(3, 4, 1))
    np.testing.assert_array_equal(oracle.physics(s1, np.full((3, 4), 9, np.int32), vertical=True), s1)


def test_vertical_sweep_is_sequential_upward():
    """One sweep over three levels: level 2 sees level 1 already updated in the same sweep
    (Fig. 1's a(k) = f(b(k), a(k-1))), which a simultaneous update would not."""
    eps = 0.01
    q0, q1, q2 = 0.9, -0.2, 0.4
    s = np.array([[[q0, q1, q2]]])
    out = oracle.physics(s, np.array([[1]], np.int32), eps, vertical=True)[0, 0]
    n1 = q1 + eps * (q0 ** 3 - q1 ** 3)
    seq2 = q2 + eps * (n1 ** 3 - q2 ** 3)
    par2 = q2 + eps * (q1 ** 3 - q2 ** 3)
    assert out[1] == pytest.approx(n1, abs=1e-16)
    assert out[2] == pytest.approx(seq2, abs=1e-16)
    assert abs(out[2] - par2) > 1e-6


def test_vertical_two_level_relaxation_rate():
    """Two levels, bottom fixed at a: the top relaxes towards a with slope 1 - 3 eps a^2
    per sweep, so a small offset d decays like d (1 - 3 eps a^2)^k."""
    a, d, k = 0.5, 1e-9, 60
    s = np.array([[[a, a + d]]])
    out = oracle.physics(s, np.array([[k]], np.int32), 0.01, vertical=True)[0, 0]
    assert out[1] - a == pytest.approx(d * (1 - 3 * 0.01 * a * a) ** k, rel=1e-5)


def test_vertical_odd_symmetric_and_bounded():
    wl = tiny(kmin=1, kmax=40, steps=3).replace(vertical=1)
    q0 = oracle.init_field(wl.nx, wl.ny, wl.nz, seed=12)
    a, _, _, _ = oracle.run(wl, q0=q0)
    b, _, _, _ = oracle.run(wl, q0=-q0)
    np.testing.assert_array_equal(a, -b)
    assert np.abs(a).max() <= 1.0
    p, _, _, _ = oracle.run(wl.replace(vertical=0), q0=q0)
    assert not np.array_equal(a, p)                   # the two physics differ


# ---------------------------------------------------------------- step order and windows
@pytest.mark.parametrize("k", [1, 5, 37])
def test_delta_field_pins_stencil_then_physics(k):
    """One step from a delta field with a uniform trip count k >= 1 (Fig. 2: the Jacobi
    kernel, then the physics kernel on its output).  Stencil first sends the delta's
    mass a to seven cells (cc*a at the centre, cn*a at the six neighbours, zero
    elsewhere since Phi(0) = 0), and the physics then maps each of those values v to
    Phi^k(v).  Physics first would give cc*Phi^k(a) and cn*Phi^k(a) instead, which
    differ for every a outside {-1, 0, 1}.  The expected values come from a scalar
    loop over Python floats (IEEE doubles), evaluated in the paper's order."""
    nx, ny, nz = 9, 8, 7
    a = 0.5
    wl = tiny(nx, ny, nz, kmin=k, kmax=k, steps=1)
    q0 = np.zeros((1, ny, nx, nz))
    cx, cy, cz = 4, 3, 3
    q0[0, cy, cx, cz] = a

    def phi_k(v):
        for _ in range(k):
            v = v + 0.01 * (v - (v * v) * v)
        return v

    want = np.zeros_like(q0)
    want[0, cy, cx, cz] = phi_k(0.4 * a)
    for dy, dx, dz in ((0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0), (0, 0, -1), (0, 0, 1)):
        want[0, cy + dy, cx + dx, cz + dz] = phi_k(0.1 * a)
    q, _, _, _ = oracle.run(wl, q0=q0)
    np.testing.assert_array_equal(q, want)
    assert want[0, cy, cx, cz] != 0.4 * phi_k(a)          # the two orders really differ


def test_delta_field_on_the_mirror_boundary():
    """A delta on the bottom level: the mirror ghost adds the cell's own value to its
    neighbour sum, so the centre gets (cc + cn)*a before the physics."""
    nx, ny, nz, k = 6, 5, 4, 3
    wl = tiny(nx, ny, nz, kmin=k, kmax=k, steps=1)
    q0 = np.zeros((1, ny, nx, nz))
    q0[0, 2, 3, 0] = 0.75

    def phi_k(v):
        for _ in range(k):
            v = v + 0.01 * (v - (v * v) * v)
        return v

    q, _, _, _ = oracle.run(wl, q0=q0)
    assert q[0, 2, 3, 0] == phi_k(0.4 * 0.75 + 0.1 * 0.75)
    assert q[0, 2, 3, 1] == phi_k(0.1 * 0.75)
    assert np.count_nonzero(q) == 6                       # centre, 4 in-plane, 1 above


def _global_slice(full, ox, oy, nxw, nyw):
    ny, nx = full.shape[-3], full.shape[-2]
    ys = (oy + np.arange(nyw)) % ny
    xs = (ox + np.arange(nxw)) % nx
    return full[..., ys, :, :][..., :, xs, :]


@pytest.mark.parametrize("ox,oy", [(-5, -4), (7, 2), (15, 13), (0, 0)])
def test_init_window_is_a_slice_of_the_field(ox, oy):
    """The windowed initial field equals the matching slice of the whole seeded field
    (local column (x, y) = global ((ox + x) mod nx, (oy + y) mod ny)), for a window that
    wraps the periodic corner and for interior windows, in every field."""
    wl = tiny(20, 16, 5, steps=1).replace(nfields=2)
    full = oracle.init_field(wl.nx, wl.ny, wl.nz, wl.seed, nfields=2)
    for f in range(2):
        win = oracle.init_window(wl, ox, oy, 11, 9, f=f)
        np.testing.assert_array_equal(win, _global_slice(full[f], ox, oy, 11, 9))


@pytest.mark.parametrize("ox,oy,hot", [
    (-5, -4, ((3, 17, 1, -1),)),                 # wraps the corner; moving hotspot
    (9, 6, ((14, 10, 2, 1), (2, 3, 0, 0))),      # interior; two hotspots
    (18, 12, ((20, 15, -1, 2),)),                # wraps both edges
])
def test_window_runner_matches_the_whole_grid(ox, oy, hot):
    """After T steps the windowed runner holds the whole-grid run's values bit for bit in
    every column at least T columns away from its border: the window is advanced as if
    it were periodic, the cost field is evaluated at global coordinates and time, and
    the 7-point update reaches one column further per step."""
    T = 3
    wl = tiny(24, 20, 6, kmin=1, kmax=20, hot=hot, sigma=3.0, steps=T)
    full, _, _, _ = oracle.run(wl)
    nxw, nyw = 14, 12
    q0 = oracle.init_window(wl, ox, oy, nxw, nyw)
    win = oracle.run_window(wl, q0, ox, oy, T)
    got = win[T:nyw - T, T:nxw - T]
    want = _global_slice(full[0], ox + T, oy + T, nxw - 2 * T, nyw - 2 * T)
    np.testing.assert_array_equal(got, want)
    # the border columns are not exact (the window's own wrap), so the interior test bites
    assert not np.array_equal(win, _global_slice(full[0], ox, oy, nxw, nyw))


def test_window_runner_honours_t0():
    """A window advanced from time t0 (a moving hotspot) equals the whole grid advanced
    t0 steps and then T more, in its interior."""
    t0, T = 4, 2
    wl = tiny(16, 14, 4, kmin=1, kmax=15, hot=((2, 12, 3, -2),), sigma=2.5, steps=t0 + T)
    full, _, _, _ = oracle.run(wl)
    mid, _, _, _ = oracle.run(wl, nsteps=t0)
    ox, oy, nxw, nyw = -3, 9, 10, 9
    q0 = _global_slice(mid[0], ox, oy, nxw, nyw)
    win = oracle.run_window(wl, q0, ox, oy, T, t0=wl.t0 + t0)
    np.testing.assert_array_equal(win[T:nyw - T, T:nxw - T],
                                  _global_slice(full[0], ox + T, oy + T, nxw - 2 * T, nyw - 2 * T))
