"""Pins of the FP64 oracle against things other than itself.

Each test compares the oracle with an independent route: the paper's printed
constant, a brute-force per-voxel intersection, numerical quadrature, Monte
Carlo detection, closed forms, or an algebraic property of EM.  A plausible
slip in the oracle (a dropped term, a wrong sign or index, a transposed
operand, a mis-scaled sigma) breaks at least one of them.
"""
import json
import os

import numpy as np
import pytest
from scipy import integrate
from scipy.special import ndtr

import oracle
import synth
from tests import brute

HERE = os.path.dirname(os.path.abspath(__file__))
C = 0.299792458


def tiny_geom(nx=8, ny=8, nz=8, v=(4.0, 4.0, 4.0), tof=300.0, R=60.0, H=40.0, origin=None, K=3.0):
    if origin is None:
        origin = (-nx * v[0] / 2, -ny * v[1] / 2, -nz * v[2] / 2)
    return dict(nx=nx, ny=ny, nz=nz, vx=v[0], vy=v[1], vz=v[2], x0=origin[0], y0=origin[1], z0=origin[2],
                scanner_radius=R, scanner_half_length=H, max_axial_angle_deg=0.0, tof_fwhm_ps=tof,
                tof_trunc_sigmas=K, c_mm_per_ps=C)


def events_through(g, n, seed, tof_sigma_ps=60.0, box_frac=0.45):
    """Random events whose lines cross the grid; short TOF blur keeps the
    TOF centre near the grid."""
    lo, hi, _, _ = brute.box(g)
    half = (hi - lo).max() * box_frac
    ev = synth.random_events_in_box(n, seed, g["scanner_radius"], g["scanner_half_length"],
                                    tof_sigma_ps=tof_sigma_ps, box=half)
    return ev.astype(np.float64)


# ------------------------------------------------------- paper constants
def test_sigma_matches_paper_value():
    gold = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))
    s = oracle.sigma_mm(gold["tof_fwhm_ps"], gold["c_mm_per_ps_implied"])
    assert round(s, gold["sigma_decimals"]) == gold["sigma_mm"]
    # with the exact speed of light the value is 19.097 mm
    assert abs(oracle.sigma_mm(300.0, C) - 19.0965) < 1e-3


# ------------------------------------------------------ projector pins
@pytest.mark.parametrize("tof", [300.0, 0.0])
@pytest.mark.parametrize("shape", [(8, 8, 8, (4.0, 4.0, 4.0)), (6, 5, 4, (3.0, 5.0, 7.0))])
def test_rows_match_bruteforce(tof, shape):
    nx, ny, nz, v = shape
    g = tiny_geom(nx, ny, nz, v, tof=tof, origin=(-9.5, -11.0, -13.0))
    ev = events_through(g, 500, seed=3 + nx)
    A = oracle.system_matrix(g, ev)
    B = brute.dense_matrix(g, ev)
    assert np.count_nonzero(B) > 2000
    scale = 1.0 if tof > 0 else np.abs(B).max()
    assert np.max(np.abs(A - B)) <= 1e-12 * scale


def test_tof_weights_match_numerical_integral():
    g = tiny_geom(tof=300.0)
    s = brute.sigma_mm(300.0, C)
    K = g["tof_trunc_sigmas"]
    ev = events_through(g, 20, seed=5)
    pdf = lambda t: np.exp(-0.5 * (t / s) ** 2) / (s * np.sqrt(2 * np.pi))
    full, _ = integrate.quad(pdf, -K * s, K * s, epsabs=1e-14)
    checked = 0
    for e in ev:
        j, a = oracle.system_row(g, e)
        mu, u = brute.ray(g, e)
        w0, w1 = brute.window(g, e)
        lo, _, v, n = brute.box(g)
        for jj, aa in zip(j, a):
            ix, iy, iz = jj % n[0], (jj // n[0]) % n[1], jj // (n[0] * n[1])
            vlo = lo + np.array([ix, iy, iz]) * v
            t0, t1 = brute._interval(vlo, vlo + v, mu, u)
            ta, tb = max(t0, w0), min(t1, w1)
            val, _ = integrate.quad(pdf, ta, tb, epsabs=1e-14)
            assert abs(aa - val / full) < 1e-11
            checked += 1
    assert checked > 100


def test_invariant_a_chord_length_nontof():
    g = tiny_geom(10, 9, 7, (4.0, 4.5, 5.0), tof=0.0)
    ev = events_through(g, 300, seed=7)
    for e in ev:
        _, a = oracle.system_row(g, e)
        L = brute.chord_length(g, e)
        assert abs(a.sum() - L) <= 1e-12 * max(L, 1.0)


def test_invariant_b_kernel_sums_to_one():
    gold = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))
    g = tiny_geom(64, 64, 64, (4.0, 4.0, 4.0), tof=300.0, R=400.0, H=200.0)
    ev = events_through(g, 400, seed=9, box_frac=0.15)
    inside = 0
    sK = g["tof_trunc_sigmas"] * brute.sigma_mm(300.0, C)
    for e in ev:
        _, a = oracle.system_row(g, e)
        mu, u = brute.ray(g, e)
        lo, hi, _, _ = brute.box(g)
        t0, t1 = brute._interval(lo, hi, mu, u)
        if t0 <= -sK and t1 >= sK:
            inside += 1
            assert abs(a.sum() - gold["kernel_weight_sum"]) < 1e-13
        else:
            s = brute.sigma_mm(300.0, C)
            ta, tb = max(t0, -sK), min(t1, sK)
            expect = max(0.0, (ndtr(tb / s) - ndtr(ta / s)) / (ndtr(3.0) - ndtr(-3.0)))
            assert abs(a.sum() - expect) < 1e-13
    assert inside > 200


def test_axis_parallel_ray_closed_form():
    g = tiny_geom(16, 8, 8, (4.0, 4.0, 4.0), tof=300.0, R=200.0, H=100.0)
    # line along +x through (y, z) = (1.3, -2.7): voxel row iy = 4, iz = 3
    y, z, dt = 1.3, -2.7, 40.0
    ev = np.array([-150.0, y, z, 150.0, y, z, dt])
    j, a = oracle.system_row(g, ev)
    s = brute.sigma_mm(300.0, C)
    mu_x = C * dt / 2.0
    planes = g["x0"] + 4.0 * np.arange(17)
    expect = {}
    for ix in range(16):
        ta = max(planes[ix] - mu_x, -3 * s)
        tb = min(planes[ix + 1] - mu_x, 3 * s)
        if tb > ta:
            expect[ix + 16 * (4 + 8 * 3)] = (ndtr(tb / s) - ndtr(ta / s)) / (ndtr(3) - ndtr(-3))
    assert sorted(j.tolist()) == sorted(expect)
    for jj, aa in zip(j, a):
        assert abs(aa - expect[jj]) < 1e-13


def test_main_diagonal_nontof():
    g = tiny_geom(8, 8, 8, (4.0, 4.0, 4.0), tof=0.0, R=200.0, H=200.0)
    ev = np.array([-100.0, -100.0, -100.0, 100.0, 100.0, 100.0, 0.0])
    j, a = oracle.system_row(g, ev)
    assert sorted(j.tolist()) == [i + 8 * (i + 8 * i) for i in range(8)]
    assert np.allclose(a, 4.0 * np.sqrt(3.0), rtol=0, atol=1e-12)


def test_endpoint_swap_symmetry():
    g = tiny_geom(8, 8, 8, tof=300.0)
    ev = events_through(g, 100, seed=11)
    sw = ev[:, [3, 4, 5, 0, 1, 2, 6]].copy()
    sw[:, 6] = -sw[:, 6]
    A = oracle.system_matrix(g, ev)
    B = oracle.system_matrix(g, sw)
    assert np.max(np.abs(A - B)) < 1e-12


def test_mirror_symmetry_x():
    g = tiny_geom(8, 6, 4, (4.0, 4.0, 4.0), tof=300.0)
    ev = events_through(g, 100, seed=13)
    mi = ev.copy()
    mi[:, 0] *= -1
    mi[:, 3] *= -1
    A = oracle.system_matrix(g, ev).reshape(-1, 4, 6, 8)
    B = oracle.system_matrix(g, mi).reshape(-1, 4, 6, 8)
    assert np.max(np.abs(A - B[..., ::-1])) < 1e-12


def test_forward_back_adjoint_and_dense():
    g = tiny_geom(8, 8, 8, tof=300.0)
    ev = events_through(g, 200, seed=17)
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, 512)
    w = rng.uniform(0, 1, 200)
    B = brute.dense_matrix(g, ev)
    f = oracle.forward(g, ev, x)
    b = oracle.back(g, ev, w)
    assert np.max(np.abs(f - B @ x)) < 1e-12 * np.abs(B @ x).max()
    assert np.max(np.abs(b - B.T @ w)) < 1e-12 * np.abs(B.T @ w).max()


# ---------------------------------------------------- sensitivity pins
def test_acceptance_centre_closed_forms():
    g1 = synth.cylinder_workload().geometry()
    assert abs(oracle.acceptance(g1, [[0, 0, 0]])[0] - 128.0 / np.hypot(128.0, 400.0)) < 1e-12
    g2 = synth.wholebody_workload().geometry()
    # atan(H/R) = 69.4 deg exceeds the 45 deg cut, so the cut decides
    assert abs(oracle.acceptance(g2, [[0, 0, 0]])[0] - np.sin(np.pi / 4)) < 1e-12


@pytest.mark.parametrize("z", [-90.0, 30.0, 110.0])
def test_acceptance_on_axis_closed_form(z):
    g = synth.cylinder_workload().geometry()
    R, H = 400.0, 128.0
    lam_hi = np.arctan(min((H - z) / R, (H + z) / R))
    lam_lo = np.arctan(max(-(H + z) / R, -(H - z) / R))
    expect = 0.5 * (np.sin(lam_hi) - np.sin(lam_lo))
    assert abs(oracle.acceptance(g, [[0, 0, z]])[0] - expect) < 1e-12


@pytest.mark.parametrize("wl", ["cylinder", "wholebody"])
def test_acceptance_matches_monte_carlo_detection(wl):
    w = synth.cylinder_workload() if wl == "cylinder" else synth.wholebody_workload()
    g = w.geometry()
    rng = np.random.default_rng(21)
    n = 400_000
    for k in range(4):
        r = rng.uniform(0, 0.9 * w.radius * 0.45)
        ph = rng.uniform(0, 2 * np.pi)
        p = [r * np.cos(ph), r * np.sin(ph), rng.uniform(-0.9, 0.9) * w.half_length]
        P = oracle.acceptance(g, [p])[0]
        acc = synth.point_source(w, p, n, seed=100 + k)
        se = np.sqrt(max(P * (1 - P), 1e-12) / n)
        assert abs(acc / n - P) < 5 * se + 2e-5, (p, acc / n, P)


def test_acceptance_quadrature_vs_adaptive():
    """2048-node midpoint rule agrees with adaptive quadrature of the same
    solid-angle integral (in lambda and phi) to 1e-6."""
    g = synth.wholebody_workload().geometry()
    R, H, lmax = 450.0, 1200.0, np.pi / 4
    for p in [(100.0, -50.0, 300.0), (250.0, 180.0, -1100.0), (0.0, 290.0, 1150.0)]:
        x, y, z = p

        def inner(phi):
            # both ends inside |z| <= H: test by direct endpoint heights
            c, s = np.cos(phi), np.sin(phi)
            b = x * c + y * s
            sq = np.sqrt(b * b - (x * x + y * y) + R * R)
            sp, sm = -b + sq, b + sq

            def ok(lam):
                t = np.tan(lam)
                return float(abs(z + sp * t) <= H and abs(z - sm * t) <= H)

            f = lambda lam: np.cos(lam) * ok(lam)
            # integrate the indicator-weighted cos over the allowed band
            val, _ = integrate.quad(f, -lmax, lmax, limit=200, points=[0.0], epsabs=1e-12)
            return val

        ref, _ = integrate.quad(inner, 0, 2 * np.pi, limit=400, epsabs=1e-11)
        ref /= 4 * np.pi
        assert abs(oracle.acceptance(g, [p])[0] - ref) < 2e-6


def test_acceptance_symmetries():
    g = synth.wholebody_workload().geometry()
    rng = np.random.default_rng(3)
    p = rng.uniform([-280, -280, -1150], [280, 280, 1150], size=(50, 3))
    a = oracle.acceptance(g, p)
    zm = p * np.array([1, 1, -1])
    rot = np.stack([-p[:, 1], p[:, 0], p[:, 2]], 1)
    assert np.max(np.abs(a - oracle.acceptance(g, zm))) < 1e-12
    assert np.max(np.abs(a - oracle.acceptance(g, rot))) < 1e-12
    # each generator of the symmetry group the whole-body parity tests use
    # to fill the sensitivity from one voxel per orbit: x and y mirrors and
    # the x <-> y swap (each maps the azimuth nodes onto themselves)
    xm = p * np.array([-1, 1, 1])
    ym = p * np.array([1, -1, 1])
    sw = p[:, [1, 0, 2]]
    for q in (xm, ym, sw):
        assert np.max(np.abs(a - oracle.acceptance(g, q))) < 1e-12


def test_sensitivity_by_orbits_equals_full_grid():
    from tests import orbits
    g = dict(nx=10, ny=10, nz=8, vx=6.0, vy=6.0, vz=7.0, x0=-30.0, y0=-30.0, z0=-28.0, scanner_radius=80.0,
             scanner_half_length=50.0, max_axial_angle_deg=45.0, tof_fwhm_ps=300.0, tof_trunc_sigmas=3.0,
             c_mm_per_ps=0.299792458)
    full = oracle.sensitivity(g, n_phi=256)
    orb = orbits.sensitivity_by_orbits(g, n_phi=256)
    assert np.max(np.abs(full - orb)) <= 1e-12 * full.max()


# ------------------------------------------------------------- EM pins
def _small_problem(seed=1, n=3000):
    g = tiny_geom(12, 12, 10, (4.0, 4.0, 4.0), tof=300.0, R=120.0, H=60.0)
    ev = events_through(g, n, seed=seed, tof_sigma_ps=100.0, box_frac=0.3)
    s = oracle.sensitivity(g, n_phi=512)
    return g, ev, s


def test_em_matches_dense_matrix_iteration():
    g, ev, s = _small_problem(n=400)
    A = brute.dense_matrix(g, ev)
    x = oracle.initial_image(g, s, len(ev))
    xo, st = oracle.mlem(g, ev, s, 4, x0=x)
    for _ in range(4):
        f = A @ x
        r = np.where(f > 0, 1.0 / np.where(f > 0, f, 1.0), 0.0)
        x = np.where(s > 0, x * (A.T @ r) / np.where(s > 0, s, 1.0), 0.0)
    assert oracle.rel_l2(xo, x) < 1e-12


def test_em_statistics_match_dense_matrix():
    """Per-iteration statistics against the brute-force matrix: the
    list-mode Poisson log-likelihood of the image fed into iteration k,
    l(x^k) = sum over events with f > 0 of log f_i - sum_j s_j x^k_j
    (Shepp & Vardi, cited in Section 2.4), N_eff and sum s x^(k+1).  The start
    image is random, so sum s x^0 differs from N and from every later sum:
    a sign slip or an off-by-one iterate in the s x term fails here."""
    g, ev, s = _small_problem(n=400)
    A = brute.dense_matrix(g, ev)
    rng = np.random.default_rng(17)
    x = np.where(s > 0, rng.uniform(0.2, 3.0, s.size), 0.0)
    assert abs(s @ x - len(ev)) > 0.05 * len(ev)
    xo, st = oracle.mlem(g, ev, s, 4, x0=x)
    for k in range(4):
        f = A @ x
        pos = f > 0
        ll = np.sum(np.log(f[pos])) - s @ x
        r = np.where(pos, 1.0 / np.where(pos, f, 1.0), 0.0)
        x = np.where(s > 0, x * (A.T @ r) / np.where(s > 0, s, 1.0), 0.0)
        assert st[k]["n_eff"] == int(pos.sum())
        assert abs(st[k]["loglik"] - ll) <= 1e-10 * abs(ll), (k, st[k]["loglik"], ll)
        assert abs(st[k]["sum_sx"] - s @ x) <= 1e-10 * abs(s @ x), k


def test_em_invariant_c_and_monotone_loglik_and_nonneg():
    g, ev, s = _small_problem()
    x, st, hist = oracle.mlem(g, ev, s, 8, history=True)
    for k in range(8):
        assert abs(st[k]["sum_sx"] - st[k]["n_eff"]) <= 1e-12 * st[k]["n_eff"]
    ll = [q["loglik"] for q in st]
    assert all(b >= a - 1e-9 * abs(a) for a, b in zip(ll, ll[1:]))
    assert np.all(hist >= 0) and np.all(np.isfinite(hist))


def test_em_single_voxel_fixed_point():
    g = tiny_geom(1, 1, 1, (8.0, 8.0, 8.0), tof=300.0, R=60.0, H=40.0)
    ev = events_through(g, 50, seed=2, box_frac=0.05)
    s = oracle.sensitivity(g, n_phi=256)
    x, st = oracle.mlem(g, ev, s, 1, x0=np.array([7.0]))
    assert abs(x[0] - st[0]["n_eff"] / s[0]) < 1e-12 * x[0]


def test_em_duplicate_and_permutation():
    g, ev, s = _small_problem(n=1000)
    x1, _ = oracle.mlem(g, ev, s, 3)
    x2, _ = oracle.mlem(g, np.concatenate([ev, ev]), s, 3)
    perm = np.random.default_rng(5).permutation(len(ev))
    x3, _ = oracle.mlem(g, ev[perm], s, 3)
    assert oracle.rel_l2(x2, 2 * x1) < 1e-12
    assert oracle.rel_l2(x3, x1) < 1e-12


def test_zero_sensitivity_voxels_stay_zero():
    g, ev, s = _small_problem(n=500)
    s = s.copy()
    s[::7] = 0.0
    x, _ = oracle.mlem(g, ev, s, 2)
    assert np.all(x[::7] == 0.0)


# --------------------------------------------------------- packed codec
def test_packed_codec_roundtrip_and_overflow():
    w = synth.wholebody_workload(n_events=20000)
    ev = synth.events(w, n=20000)
    p = oracle.pack_events(ev)
    d = oracle.decode_packed(p)
    # half a quantum, plus the FP32 rounding of x * 10 (|x * 10| < 2^14)
    assert np.max(np.abs(d[:, :6] - ev[:, :6])) <= 0.05 + 2.0 ** -10 / 10
    rel = np.abs(d[:, 6] - ev[:, 6]) / np.maximum(np.abs(ev[:, 6]), 1e-3)
    assert np.max(rel[np.abs(ev[:, 6]) > 1.0]) <= 2.0 ** -11
    bad = ev[:2].copy()
    bad[0, 2] = 3300.0
    with pytest.raises(OverflowError):
        oracle.pack_events(bad)


# ---- median sieve between iterations (Section 2.4)

def _median_brute(a, x, y, z):
    """The 14th smallest of the 27 neighbours of voxel (x, y, z), 0 outside."""
    nz, ny, nx = a.shape
    vals = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                i, j, k = x + dx, y + dy, z + dz
                inside = 0 <= i < nx and 0 <= j < ny and 0 <= k < nz
                vals.append(float(a[k, j, i]) if inside else 0.0)
    return sorted(vals)[13]


@pytest.mark.parametrize("shape", [(5, 4, 3), (1, 1, 1), (2, 1, 3), (6, 5, 4)])
def test_median3_matches_bruteforce(shape):
    nx, ny, nz = shape
    a = np.random.default_rng(7).uniform(0.0, 1.0, (nz, ny, nx)).astype(np.float32)
    a[a < 0.2] = 0.0  # ties with the zero border
    got = oracle.median3(a.reshape(-1), nx, ny, nz).reshape(nz, ny, nx)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                assert got[z, y, x] == _median_brute(a, x, y, z)


def test_median3_constant_image_border_counts():
    """Constant c on 5^3: inside and on faces (18 or 27 neighbours in the grid,
    at most 9 zeros) the median is c; on edges (12 in the grid) and corners (8)
    the 15 or 19 zeros win."""
    c = 2.5
    m = oracle.median3(np.full(125, c), 5, 5, 5).reshape(5, 5, 5)
    for z in range(5):
        for y in range(5):
            for x in range(5):
                on = sum(v in (0, 4) for v in (x, y, z))
                assert m[z, y, x] == (c if on <= 1 else 0.0)


def test_median3_removes_impulse_and_keeps_linear_ramp():
    a = np.zeros((7, 7, 7))
    a[3, 3, 3] = 100.0
    assert not oracle.median3(a.reshape(-1), 7, 7, 7).any()
    # a linear function is symmetric about each interior voxel: the median is the centre value
    z, y, x = np.meshgrid(np.arange(7), np.arange(7), np.arange(7), indexing="ij")
    r = (1.0 * x + 3.0 * y + 9.0 * z + 1.0)  # distinct values, odd symmetric neighbourhoods
    m = oracle.median3(r.reshape(-1), 7, 7, 7).reshape(7, 7, 7)
    assert np.array_equal(m[1:-1, 1:-1, 1:-1], r[1:-1, 1:-1, 1:-1])


# ---- TOF scatter rejection (Section 2.2)

def _box_geom(n=20, v=4.0, fwhm=300.0):
    return dict(nx=n, ny=n, nz=n, vx=v, vy=v, vz=v, x0=-n * v / 2, y0=-n * v / 2, z0=-n * v / 2,
                scanner_radius=400.0, scanner_half_length=400.0, max_axial_angle_deg=0.0, tof_fwhm_ps=fwhm,
                tof_trunc_sigmas=3.0, c_mm_per_ps=0.299792458)


def test_tof_keep_axis_ray_threshold_closed_form():
    """A body of one 4 mm voxel at the grid centre, an x-axis LOR through it,
    the TOF centre d mm before the voxel's near face: kept iff d < 1.96 sigma
    (sigma = 19.11 mm at 300 ps: the paper's value)."""
    g = _box_geom()
    mask = np.zeros(20 ** 3, np.uint8)
    mask[(10 * 20 + 10) * 20 + 10] = 1  # voxel [0, 4) mm on every axis
    sig = oracle.sigma_mm(300.0)
    c = 0.299792458
    evs = []
    for d in (1.959964 * sig - 0.5, 1.959964 * sig + 0.5):
        xc = 0.0 - d  # centre on the x axis, d before the face x = 0
        # mu = mid + (c dt / 2) u with u = +x, mid = 0: dt = 2 xc / c
        evs.append([-400.0, 2.0, 2.0, 400.0, 2.0, 2.0, 2.0 * xc / c])
    keep = oracle.tof_keep(g, np.array(evs), mask)
    assert keep.tolist() == [True, False]


def test_tof_keep_full_and_empty_masks():
    g = _box_geom()
    c = 0.299792458
    sig = oracle.sigma_mm(300.0)
    # centres on the x axis at 0 (inside), 40 + 1.9 sigma (interval reaches the box), 40 + 2.1 sigma (misses)
    xs = [0.0, 40.0 + 1.9 * sig, 40.0 + 2.1 * sig]
    evs = np.array([[-400.0, 1.0, 1.0, 400.0, 1.0, 1.0, 2.0 * x / c] for x in xs])
    assert oracle.tof_keep(g, evs, np.ones(20 ** 3)).tolist() == [True, True, False]
    assert not oracle.tof_keep(g, evs, np.zeros(20 ** 3)).any()


def test_tof_keep_matches_dense_sampling():
    """Against a dense point sampler (0.01 mm steps along the stretch, a
    different method from the crossing walk) on random LORs and a random
    blob mask; events whose masked stretch is shorter than 0.05 mm, or that
    change with the stretch end moved by 0.05 mm, may go either way."""
    g = _box_geom(n=12)
    rng = np.random.default_rng(21)
    mask = (rng.uniform(size=12 ** 3) < 0.08).astype(np.uint8)
    n = 300
    a = rng.normal(size=(n, 3))
    a /= np.linalg.norm(a, axis=1)[:, None]
    p0 = rng.uniform(-24, 24, size=(n, 3))
    evs = np.concatenate([p0 - 300 * a, p0 + 300 * a, rng.normal(0, 150, (n, 1))], axis=1)
    keep = oracle.tof_keep(g, evs, mask)
    strict = oracle.tof_keep(g, evs, mask, grow=-0.05, min_piece=0.05)
    loose = oracle.tof_keep(g, evs, mask, grow=0.05)
    sig = oracle.sigma_mm(300.0)
    half = oracle.TOF_REJECT_Z * sig
    c = 0.299792458
    m = mask.reshape(12, 12, 12)
    for i in range(n):
        d = evs[i, 3:6] - evs[i, :3]
        u = d / np.linalg.norm(d)
        mu = 0.5 * (evs[i, :3] + evs[i, 3:6]) + c * evs[i, 6] / 2 * u
        ts = np.arange(-half, half, 0.01)
        pts = mu + ts[:, None] * u
        idx = np.floor((pts + 24.0) / 4.0).astype(int)
        ok = np.all((idx >= 0) & (idx < 12), axis=1)
        hit = bool(m[idx[ok, 2], idx[ok, 1], idx[ok, 0]].any()) if ok.any() else False
        assert strict[i] <= hit <= loose[i], i
        assert strict[i] <= keep[i] <= loose[i], i
    assert 20 < keep.sum() < n - 20  # both outcomes occur


# ---- attenuation weights on the LOR (Section 2.4)

def test_attenuation_factor_closed_form():
    """A uniform mu over the grid: the factor is exp(mu x chord length), the
    chord through the box in closed form for an axis-parallel LOR."""
    g = _box_geom(n=10, v=4.0)
    mu = np.full(1000, 0.0096)  # water at 511 keV, 1/mm
    ev = np.array([[-300.0, 1.0, 2.0, 300.0, 1.0, 2.0, 0.0],     # along x: 40 mm inside
                   [1.0, 1.0, -300.0, 1.0, 1.0, 300.0, 50.0],    # along z: 40 mm
                   [-300.0, 30.0, 0.0, 300.0, 30.0, 0.0, 0.0]])  # misses the grid: factor 1
    acf = oracle.attenuation_factors(g, ev, mu)
    assert np.allclose(acf, [np.exp(0.0096 * 40), np.exp(0.0096 * 40), 1.0], rtol=1e-12)


def test_weighted_mlem_unit_weights_duplicates_and_normalisation():
    """Unit weights reproduce the plain MLEM; weight 2 on an event equals
    loading it twice; sum_j s_j x_j after an iteration equals the weight sum
    over events with (A x)_i > 0."""
    g = _box_geom(n=6, v=4.0)
    rng = np.random.default_rng(31)
    a = rng.normal(size=(40, 3))
    a /= np.linalg.norm(a, axis=1)[:, None]
    p0 = rng.uniform(-8, 8, size=(40, 3))
    ev = np.concatenate([p0 - 300 * a, p0 + 300 * a, rng.normal(0, 40, (40, 1))], axis=1)
    s = rng.uniform(0.5, 1.5, 216)
    x0 = np.full(216, 0.3)
    x1, _ = oracle.mlem(g, ev, s, 2, x0=x0)
    assert np.allclose(oracle.mlem_weighted(g, ev, s, 2, np.ones(40), x0), x1, rtol=1e-12, atol=0)
    w = np.ones(40)
    w[:5] = 2.0
    xd, _ = oracle.mlem(g, np.concatenate([ev, ev[:5]]), s, 2, x0=x0)
    assert np.allclose(oracle.mlem_weighted(g, ev, s, 2, w, x0), xd, rtol=1e-12, atol=0)
    wr = rng.uniform(0.5, 3.0, 40)
    xw = oracle.mlem_weighted(g, ev, s, 1, wr, x0)
    f = oracle.forward(g, ev, x0)
    assert abs((s * xw).sum() - wr[f > 0].sum()) < 1e-10 * wr.sum()


# ---- the paper's sampled TOF projector (Section 2.3)

def _random_lors(n, seed, spread=8.0, tof=40.0):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n, 3))
    a /= np.linalg.norm(a, axis=1)[:, None]
    p0 = rng.uniform(-spread, spread, size=(n, 3))
    return np.concatenate([p0 - 300 * a, p0 + 300 * a, rng.normal(0, tof, (n, 1))], axis=1)


def test_sampled_weights_and_uniform_image():
    """Weights sum to 1; a uniform image inside a grid holding the whole
    +-3 sigma window gives f = 1 (the sampled form of invariant (b))."""
    g = _box_geom(n=40, v=4.0)
    idx, w, _ = oracle.sampled_system(g, _random_lors(50, 41, spread=5.0, tof=20.0))
    assert abs(w.sum() - 1.0) < 1e-15 and np.allclose(w, w[::-1])
    assert np.all(idx >= 0)
    f = oracle.sampled_forward(g, _random_lors(50, 41, spread=5.0, tof=20.0), np.ones(40 ** 3))
    assert np.allclose(f, 1.0, rtol=1e-14)


def test_sampled_adjoint_and_endpoint_swap():
    g = _box_geom(n=12, v=4.0)
    ev = _random_lors(200, 42)
    rng = np.random.default_rng(43)
    x, r = rng.uniform(size=12 ** 3), rng.uniform(size=200)
    assert np.isclose(oracle.sampled_forward(g, ev, x) @ r, x @ oracle.sampled_back(g, ev, r), rtol=1e-12)
    sw = np.concatenate([ev[:, 3:6], ev[:, :3], -ev[:, 6:7]], axis=1)
    idx_a, _, near_a = oracle.sampled_system(g, ev)
    idx_b, _, _ = oracle.sampled_system(g, sw)
    ok = near_a.min(axis=1) > 1e-6  # away from planes the swapped event samples the same points, reversed
    assert np.array_equal(np.sort(idx_a[ok], axis=1), np.sort(idx_b[ok], axis=1))


def test_sampled_converges_to_exact_integral():
    """With many samples the sampled projector tends to the exact per-piece
    integral of the oracle's main projector (same centre, direction and
    window conventions)."""
    g = _box_geom(n=16, v=4.0)
    ev = _random_lors(30, 44, spread=6.0, tof=30.0)
    x = np.random.default_rng(45).uniform(0.5, 1.5, 16 ** 3)
    idx, w, _ = oracle.sampled_system(g, ev, n_samples=40000)
    f_many = np.sum(np.where(idx >= 0, w * x[np.maximum(idx, 0)], 0.0), axis=1)
    f_exact = oracle.forward(g, ev, x)
    # the exact kernel is normalised over the truncated window; so are the sample weights
    assert np.allclose(f_many, f_exact, rtol=2e-3)
