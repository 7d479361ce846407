"""Pins of the FP64 oracle against facts it does not compute itself.

The paper prints no worked numerical example of a projection, so every pin
is a closed form, an invariant, a textbook special case or an independent
brute-force formulation (tests/brute.py).  Each test says which mistake it
would catch.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import special, stats

import oracle
from brute import gauss_matrix, system_matrix, tof_weight_quadrature

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


from helpers import f32, random_rays, tofd  # noqa: E402


# ---------------------------------------------------------------- closed forms

def test_axis_aligned_uniform_chord():
    """Pin 1: a ray along an axis through a uniform image of value 1 gives n_p * h_p
    (ray length inside the slab between the outer voxel centres' planes, one voxel per plane).
    Catches a wrong incidence-angle factor, a dropped plane, or an off-by-one in the plane loop."""
    dim = (7, 5, 4)
    vs = (1.5, 2.0, 2.5)
    origin = (-4.5, -4.0, -3.75)
    img = np.ones(dim)
    for p in range(3):
        inplane = [a for a in range(3) if a != p]
        xs = np.zeros((1, 3), np.float32)
        xe = np.zeros((1, 3), np.float32)
        xs[0, p], xe[0, p] = -100.0, 100.0
        for a in inplane:  # an in-plane point strictly inside the centre hull
            xs[0, a] = xe[0, a] = origin[a] + 0.37 * vs[a] * (dim[a] - 1)
        val = oracle.fwd(xs, xe, origin, vs, dim, img)[0]
        assert val == pytest.approx(dim[p] * vs[p], rel=1e-14)
        # reversed direction
        val2 = oracle.fwd(xe, xs, origin, vs, dim, img)[0]
        assert val2 == pytest.approx(dim[p] * vs[p], rel=1e-14)


def test_affine_image_exact():
    """Pin 2: bilinear interpolation reproduces affine images and the plane sum is a
    midpoint rule, so for x_v = a + b.c_v and a ray inside the centre hull,
    p = n_p * ell * (a + b . X(t_mid)), X(t_mid) the ray point on the middle plane.
    Catches a wrong interpolation weight, a transposed in-plane axis, or a wrong ell."""
    rng = np.random.default_rng(11)
    dim = (9, 8, 7)
    vs = (1.25, 2.0, 1.5)
    origin = (3.0, -7.0, 1.0)
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in dim], indexing="ij"), -1)
    centres = np.asarray(origin) + idx * np.asarray(vs)
    alpha, beta = 2.5, np.array([0.3, -0.7, 1.1])
    img = alpha + centres @ beta
    lo = np.asarray(origin)
    hi = lo + (np.asarray(dim) - 1) * np.asarray(vs)
    for trial in range(40):
        p = trial % 3
        inplane = [a for a in range(3) if a != p]
        s = np.zeros(3)
        e = np.zeros(3)
        s[p], e[p] = lo[p] - 30.0, hi[p] + 30.0
        if trial % 2:
            s[p], e[p] = e[p], s[p]
        # in-plane coordinates chosen so that the whole chord between the outer planes stays in the hull
        for a in inplane:
            a0, a1 = rng.uniform(lo[a] + 0.1 * (hi[a] - lo[a]), hi[a] - 0.1 * (hi[a] - lo[a]), size=2)
            # extend linearly to the endpoints, keeping the slope small enough to stay principal
            tlo = (lo[p] - s[p]) / (e[p] - s[p])
            thi = (hi[p] - s[p]) / (e[p] - s[p])
            slope = (a1 - a0) / (thi - tlo)
            s[a] = a0 - slope * tlo
            e[a] = a0 + slope * (1.0 - tlo)
        xs = s.astype(np.float32)[None]
        xe = e.astype(np.float32)[None]
        d = xe[0].astype(float) - xs[0].astype(float)
        if np.argmax(np.abs(d)) != p:
            continue
        ell = vs[p] * np.linalg.norm(d) / abs(d[p])
        zmid = lo[p] + 0.5 * (dim[p] - 1) * vs[p]
        tmid = (zmid - xs[0, p]) / d[p]
        X = xs[0].astype(float) + tmid * d
        expect = dim[p] * ell * (alpha + X @ beta)
        got = oracle.fwd(xs, xe, origin, vs, dim, img)[0]
        assert got == pytest.approx(expect, rel=1e-12)


def test_gaussian_blob_converges_to_line_integral():
    """Pin 9: for a smooth blob, Joseph's sum approaches the continuous line integral
    (closed form for a Gaussian: tau sqrt(2 pi) exp(-dist^2 / (2 tau^2))) with O(h^2)
    error.  Catches any error in the ell normalisation that a self-consistent test cannot."""
    tau = 6.0
    c = np.array([1.3, -0.7, 0.4])
    rng = np.random.default_rng(5)
    dirs = rng.normal(size=(6, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    offs = rng.normal(size=(6, 3)) * 3.0
    errs = []
    for h in (2.0, 1.0, 0.5):
        n = int(round(80.0 / h)) + 1
        dim = (n, n, n)
        origin = tuple(-0.5 * (n - 1) * h for _ in range(3))
        ax = origin[0] + h * np.arange(n)
        X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
        img = np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2 * tau * tau))
        xs = (offs + 150.0 * dirs).astype(np.float32)
        xe = (offs - 150.0 * dirs).astype(np.float32)
        got = oracle.fwd(xs, xe, origin, (h, h, h), dim, img)
        d = xe.astype(float) - xs.astype(float)
        u = d / np.linalg.norm(d, axis=1, keepdims=True)
        w = c - xs.astype(float)
        dist2 = np.sum(w * w, 1) - np.sum(w * u, 1) ** 2
        exact = tau * math.sqrt(2 * math.pi) * np.exp(-dist2 / (2 * tau * tau))
        errs.append(np.max(np.abs(got - exact) / exact))
    assert errs[-1] < 2e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0  # second order


# ------------------------------------------------------------- brute force

GRIDS = [
    ((5, 4, 3), (1.0, 1.5, 2.0), (-2.0, -2.25, -2.0)),
    ((3, 6, 4), (2.0, 1.0, 1.25), (0.5, -3.0, 1.0)),
]


@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_nontof_matches_bruteforce(gi):
    """Pin 3 (non-TOF): oracle fwd and back == independent tent-function system matrix.
    Covers all principal axes, both directions, rays missing or grazing the grid and
    endpoints inside the grid (segment semantics).  Catches index, sign and transposition errors."""
    dim, vs, origin = GRIDS[gi]
    rng = np.random.default_rng(100 + gi)
    xs, xe = random_rays(rng, 60, origin, vs, dim, inside_frac=0.25)
    # add exact 45-degree ties and axis-aligned rays along voxel-centre lines (stencil edge cases)
    extra_s = np.array([[-20, -20, 0.3], [-20, 0.1, -20], [0.5, -20, -20], [-20, origin[1], origin[2]],
                        [origin[0] + vs[0] * (dim[0] - 1), -20, origin[2] + vs[2] * (dim[2] - 1)]], np.float32)
    extra_e = np.array([[20, 20, 0.3], [20, 0.1, 20], [0.5, 20, 20], [20, origin[1], origin[2]],
                        [origin[0] + vs[0] * (dim[0] - 1), 20, origin[2] + vs[2] * (dim[2] - 1)]], np.float32)
    xs = np.concatenate([xs, extra_s])
    xe = np.concatenate([xe, extra_e])
    A = system_matrix(xs, xe, origin, vs, dim)
    x = rng.uniform(0, 1, size=dim)
    y = rng.uniform(0, 1, size=xs.shape[0])
    np.testing.assert_allclose(oracle.fwd(xs, xe, origin, vs, dim, x), A @ x.ravel(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.back(xs, xe, origin, vs, dim, y).ravel(), A.T @ y, rtol=1e-12, atol=1e-12)
    assert np.count_nonzero(A.sum(1)) > 40  # most rays do hit the grid


@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_tof_matches_bruteforce(gi):
    """Pin 3 (TOF sinogram and listmode): oracle == brute force whose TOF weights come from
    quadrature of the truncated Gaussian over each bin (no erf).  Catches a wrong bin centre,
    sign of the TOF coordinate, sigma scaling or truncation."""
    dim, vs, origin = GRIDS[gi]
    rng = np.random.default_rng(200 + gi)
    xs, xe = random_rays(rng, 30, origin, vs, dim, inside_frac=0.2)
    tof = tofd(bin_width=2.5, sigma=1.7, n_sigmas=2.5, n_bins=9, center_offset=0.4)
    A = system_matrix(xs, xe, origin, vs, dim, tof=tof, mode="sino")
    x = rng.uniform(0, 1, size=dim)
    y = rng.uniform(0, 1, size=(xs.shape[0], tof["n_bins"]))
    np.testing.assert_allclose(oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tof, x),
                               np.einsum("lbv,v->lb", A, x.ravel()), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(oracle.back_tof_sino(xs, xe, origin, vs, dim, tof, y).ravel(),
                               np.einsum("lbv,lb->v", A, y), rtol=1e-11, atol=1e-12)
    bins = rng.integers(-1, tof["n_bins"] + 1, size=xs.shape[0]).astype(np.int16)  # incl. out of range
    Alm = system_matrix(xs, xe, origin, vs, dim, tof=tof, mode="lm", bins=bins)
    ylm = rng.uniform(0, 1, size=xs.shape[0])
    np.testing.assert_allclose(oracle.fwd_tof_lm(xs, xe, origin, vs, dim, tof, bins, x), Alm @ x.ravel(),
                               rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(oracle.back_tof_lm(xs, xe, origin, vs, dim, tof, bins, ylm).ravel(),
                               Alm.T @ ylm, rtol=1e-11, atol=1e-12)


def test_count_samples_bruteforce():
    """The work counter: planes on the segment whose 2x2 stencil has a neighbour in the grid."""
    dim, vs, origin = GRIDS[0]
    rng = np.random.default_rng(7)
    xs, xe = random_rays(rng, 50, origin, vs, dim, inside_frac=0.2)
    tot, per = oracle.count_samples(xs, xe, origin, vs, dim, per_ray=True)
    for l in range(xs.shape[0]):
        d32 = (xe[l] - xs[l]).astype(np.float32)
        p = int(np.argmax(np.abs(d32)))
        inplane = [a for a in range(3) if a != p]
        cnt = 0
        for k in range(dim[p]):
            t = (origin[p] + k * vs[p] - float(xs[l, p])) / (float(xe[l, p]) - float(xs[l, p]))
            if t < 0 or t > 1:
                continue
            X = xs[l].astype(float) + t * (xe[l].astype(float) - xs[l].astype(float))
            idx = [(X[a] - origin[a]) / vs[a] for a in inplane]
            ok = all(math.floor(i) + 1 >= 0 and math.floor(i) <= dim[a] - 1 for i, a in zip(idx, inplane))
            cnt += ok
        assert per[l] == cnt
    assert tot == per.sum()


# ---------------------------------------------------------------- invariants

def test_adjoint_identity_all_variants():
    """Pin 4: <A x, y> == <x, A^T y> in fp64 for the three variants."""
    rng = np.random.default_rng(3)
    dim, vs, origin = (12, 10, 6), (2.0, 2.0, 3.0), (-11.0, -9.0, -7.5)
    xs, xe = random_rays(rng, 400, origin, vs, dim, inside_frac=0.1)
    tof = tofd(6.0, 5.0, 3.0, 11)
    x = rng.uniform(size=dim)
    y = rng.uniform(size=xs.shape[0])
    ys = rng.uniform(size=(xs.shape[0], 11))
    bins = rng.integers(0, 11, size=xs.shape[0]).astype(np.int16)
    pairs = [
        (oracle.fwd(xs, xe, origin, vs, dim, x), y, oracle.back(xs, xe, origin, vs, dim, y)),
        (oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tof, x), ys, oracle.back_tof_sino(xs, xe, origin, vs, dim, tof, ys)),
        (oracle.fwd_tof_lm(xs, xe, origin, vs, dim, tof, bins, x), y,
         oracle.back_tof_lm(xs, xe, origin, vs, dim, tof, bins, y)),
    ]
    for Ax, yy, ATy in pairs:
        lhs = float(np.sum(Ax * yy))
        rhs = float(np.sum(x * ATy))
        assert lhs == pytest.approx(rhs, rel=1e-12)
        assert lhs > 0


def test_tof_bin_sum_reproduces_nontof():
    """Pin 5: for a LOR whose samples all lie well inside the TOF bin range, the TOF weights
    telescope: sum_t p_t = erf(n_sigmas / sqrt(2)) * p_nonTOF (not renormalised truncation).
    With n_sigmas = 8 the factor is 1 - 1.2e-15."""
    rng = np.random.default_rng(4)
    dim, vs, origin = (20, 18, 8), (2.0, 2.0, 2.0), (-19.0, -17.0, -7.0)
    xs, xe = random_rays(rng, 50, origin, vs, dim)
    x = rng.uniform(size=dim)
    pn = oracle.fwd(xs, xe, origin, vs, dim, x)
    for nsig, factor in ((3.0, special.erf(3.0 / math.sqrt(2.0))), (8.0, 1.0)):
        tof = tofd(4.0, 3.0, nsig, 41)  # bins cover +-82 mm, samples lie within ~40 mm
        pt = oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tof, x)
        factor = special.erf(f32(nsig) * f32(3.0) / (math.sqrt(2.0) * f32(3.0)))
        np.testing.assert_allclose(pt.sum(1), factor * pn, rtol=1e-13, atol=1e-13)
    with open(os.path.join(GOLDEN, "closed_forms.json")) as fh:
        gold = json.load(fh)
    assert special.erf(3.0 / math.sqrt(2.0)) == pytest.approx(gold["tof_mass_3sigma"]["value"], rel=1e-15)


def test_single_voxel_textbook_tof_weight():
    """Pin 6: one hot voxel on an axis-aligned ray through its centre gives
    p_t = ell * w_t(s) with w_t the Gaussian-cdf difference over the bin (scipy's normal cdf),
    for bins where the truncation does not bite.  Catches a wrong TOF coordinate origin or sign."""
    dim, vs, origin = (21, 3, 3), (2.0, 2.0, 2.0), (-20.0, -2.0, -2.0)
    img = np.zeros(dim)
    img[15, 1, 1] = 1.0  # centre at x = +10 mm
    xs = np.array([[-60.0, 0.0, 0.0]], np.float32)
    xe = np.array([[40.0, 0.0, 0.0]], np.float32)  # midpoint x = -10, so s = +20 mm
    tof = tofd(5.0, 4.0, 6.0, 15)
    pt = oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tof, img)[0]
    s = 20.0
    for t in range(15):
        c = (t - 7) * 5.0
        if abs(s - c) + 2.5 < 6.0 * 4.0 - 1e-9:
            expect = 2.0 * (stats.norm.cdf((s - c + 2.5) / 4.0) - stats.norm.cdf((s - c - 2.5) / 4.0))
            assert pt[t] == pytest.approx(expect, rel=1e-12, abs=1e-15)
    # integral of the kernel over s equals bin width * truncated mass (pin of the convolution)
    grid = np.linspace(-40, 40, 8001)
    w = np.array([tof_weight_quadrature(si, 0.0, 5.0, 4.0, 3.0) for si in grid])
    assert np.trapezoid(w, grid) == pytest.approx(5.0 * special.erf(3.0 / math.sqrt(2)), rel=1e-6)


def test_listmode_equals_sinogram_bin():
    """Pin 7: TOF listmode projection of bin t is bit-identical to column t of the sinogram
    projection, and listmode back projection to the sinogram back projection of that column."""
    rng = np.random.default_rng(8)
    dim, vs, origin = (10, 9, 5), (2.0, 2.0, 2.0), (-9.0, -8.0, -4.0)
    xs, xe = random_rays(rng, 80, origin, vs, dim)
    tof = tofd(3.0, 2.5, 3.0, 13)
    x = rng.uniform(size=dim)
    sino = oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tof, x)
    y = rng.uniform(size=xs.shape[0])
    for t in (0, 5, 12):
        bins = np.full(xs.shape[0], t, np.int16)
        assert np.array_equal(oracle.fwd_tof_lm(xs, xe, origin, vs, dim, tof, bins, x), sino[:, t])
        ys = np.zeros((xs.shape[0], 13))
        ys[:, t] = y
        np.testing.assert_allclose(oracle.back_tof_lm(xs, xe, origin, vs, dim, tof, bins, y),
                                   oracle.back_tof_sino(xs, xe, origin, vs, dim, tof, ys), rtol=1e-15, atol=0)
    # out-of-range listmode bins contribute nothing
    bad = np.array([-1, 13, 200, -32768] * 20, np.int16)[: xs.shape[0]]
    assert not np.any(oracle.fwd_tof_lm(xs, xe, origin, vs, dim, tof, bad, x))


def test_symmetries():
    """Pin 8: swapping start/end leaves non-TOF unchanged and mirrors TOF bins (offset 0);
    a joint translation of rays and grid, and a joint permutation of coordinate and image axes,
    leave every variant unchanged."""
    rng = np.random.default_rng(9)
    dim, vs, origin = (11, 9, 7), (2.0, 1.5, 2.5), (-10.0, -6.0, -7.5)
    # coordinates on a 1/64 mm lattice so that the translated inputs stay exact in float32
    xs, xe = random_rays(rng, 120, origin, vs, dim, grid_step=1.0 / 64)
    tof = tofd(3.0, 2.0, 3.0, 15)
    x = rng.uniform(size=dim)
    p = oracle.fwd(xs, xe, origin, vs, dim, x)
    np.testing.assert_allclose(oracle.fwd(xe, xs, origin, vs, dim, x), p, rtol=1e-13)
    pt = oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tof, x)
    np.testing.assert_allclose(oracle.fwd_tof_sino(xe, xs, origin, vs, dim, tof, x), pt[:, ::-1], rtol=1e-12,
                               atol=1e-14)
    shift = np.array([37.0, -12.0, 5.0], np.float32)
    o2 = tuple(np.asarray(origin) + shift)
    np.testing.assert_allclose(oracle.fwd(xs + shift, xe + shift, o2, vs, dim, x), p, rtol=1e-12)
    np.testing.assert_allclose(oracle.fwd_tof_sino(xs + shift, xe + shift, o2, vs, dim, tof, x), pt, rtol=1e-11,
                               atol=1e-13)
    perm = (2, 0, 1)
    xsP, xeP = xs[:, perm].copy(), xe[:, perm].copy()
    dimP = tuple(dim[a] for a in perm)
    vsP = tuple(vs[a] for a in perm)
    oP = tuple(origin[a] for a in perm)
    xP = np.ascontiguousarray(np.transpose(x, perm))
    np.testing.assert_allclose(oracle.fwd(xsP, xeP, oP, vsP, dimP, xP), p, rtol=1e-12)
    np.testing.assert_allclose(oracle.fwd_tof_sino(xsP, xeP, oP, vsP, dimP, tof, xP), pt, rtol=1e-11, atol=1e-13)
    y = rng.uniform(size=xs.shape[0])
    bP = oracle.back(xsP, xeP, oP, vsP, dimP, y)
    np.testing.assert_allclose(np.transpose(bP, np.argsort(perm)), oracle.back(xs, xe, origin, vs, dim, y),
                               rtol=1e-12, atol=1e-14)


def test_degenerate_rays():
    """Zero-length and non-finite rays contribute nothing; a ray missing the grid gives 0."""
    dim, vs, origin = (4, 4, 4), (1.0, 1.0, 1.0), (-1.5, -1.5, -1.5)
    x = np.ones(dim)
    xs = np.array([[1, 1, 1], [np.nan, 0, 0], [-50, 30, 0], [0, 0, np.inf]], np.float32)
    xe = np.array([[1, 1, 1], [5, 0, 0], [50, 30, 0], [0, 0, 5]], np.float32)
    assert not np.any(oracle.fwd(xs, xe, origin, vs, dim, x))
    assert not np.any(oracle.back(xs, xe, origin, vs, dim, np.ones(4)))
    assert oracle.fwd(xs[:0], xe[:0], origin, vs, dim, x).shape == (0,)


# ---------------------------------------------------------------------- OSEM

def _osem_problem(seed=12, n_ev=300):
    rng = np.random.default_rng(seed)
    dim, vs, origin = (6, 5, 4), (2.0, 2.0, 2.0), (-5.0, -4.0, -3.0)
    xs, xe = random_rays(rng, n_ev, origin, vs, dim)
    tof = tofd(3.0, 2.5, 3.0, 9)
    bins = rng.integers(2, 7, size=n_ev).astype(np.int16)
    # sensitivity from a separate "scanner" ray set
    ss, se = random_rays(np.random.default_rng(seed + 1), 2000, origin, vs, dim)
    sens = oracle.back(ss, se, origin, vs, dim, np.ones(ss.shape[0]))
    return xs, xe, bins, dim, vs, origin, tof, sens


def test_osem_matches_dense_algebra():
    """The OSEM oracle equals the same update written with the brute-force matrix and numpy
    algebra: x <- x * A_j^T (1 / (A_j x + bg)) / (sens / n_sub), zero where sens == 0."""
    xs, xe, bins, dim, vs, origin, tof, sens = _osem_problem()
    sens = sens.copy()
    sens.ravel()[::7] = 0.0  # some voxels without sensitivity
    A = system_matrix(xs, xe, origin, vs, dim, tof=tof, mode="lm", bins=bins)
    bg, n_iter, n_sub = 0.1, 2, 3
    x = (sens > 0).astype(float).ravel()
    s = sens.ravel()
    for _ in range(n_iter):
        for j in range(n_sub):
            Aj = A[j::n_sub]
            ybar = Aj @ x + bg
            acc = Aj.T @ (1.0 / ybar)
            x = np.where(s > 0, x * acc / np.where(s > 0, s / n_sub, 1.0), 0.0)
    got = oracle.lm_osem(xs, xe, bins, origin, vs, dim, tof, sens, bg, n_iter, n_sub, (sens > 0).astype(float))
    np.testing.assert_allclose(got.ravel(), x, rtol=1e-11, atol=1e-14)
    assert np.all(got >= 0) and np.all(got.ravel()[s == 0] == 0)


def test_osem_count_conservation():
    """Pin 10: with zero background, one EM update satisfies sum_v sens_v x_v^new = number of
    events with positive expectation a_e . x (exact invariant of the multiplicative update),
    for a flat and for a random positive starting image."""
    xs, xe, bins, dim, vs, origin, tof, sens = _osem_problem(seed=21, n_ev=400)
    rng = np.random.default_rng(22)
    for x0 in ((sens > 0).astype(float), rng.uniform(0.5, 2.0, size=dim) * (sens > 0)):
        one = oracle.lm_osem(xs, xe, bins, origin, vs, dim, tof, sens, 0.0, 1, 1, x0)
        ybar = oracle.fwd_tof_lm(xs, xe, origin, vs, dim, tof, bins, x0)
        n_pos = int(np.count_nonzero(ybar > 0))
        assert n_pos > 300
        assert float(np.sum(sens * one)) == pytest.approx(n_pos, rel=1e-12)


# ------------------------------------------------------- resolution model

FWHM_RES = 4.5  # mm, the paper's image-based resolution model (Sec. 2.6)


def test_gauss_matches_scipy():
    """Pin 11: the blur equals scipy.ndimage.gaussian_filter with sigma = FWHM / (2 sqrt(2 ln 2)) / h
    per axis, zero ('constant') boundary and truncation at 4 sigma (an independent library
    routine).  Catches a wrong FWHM->sigma conversion, a wrong radius, a transposed axis/voxel
    size pairing or non-zero boundary handling."""
    from scipy import ndimage

    rng = np.random.default_rng(31)
    for dim, vs, fw in (((17, 13, 11), (1.65, 1.65, 2.0), 4.5), ((9, 12, 15), (2.78, 2.0, 1.0), (4.5, 3.0, 6.0))):
        x = rng.uniform(0, 1, size=dim)
        got = oracle.gauss3d(x, vs, fw)
        sig = np.broadcast_to(np.asarray(fw, float), (3,)) / math.sqrt(8 * math.log(2)) / np.asarray(vs, np.float32)
        want = ndimage.gaussian_filter(x, sigma=sig, mode="constant", cval=0.0, truncate=4.0)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)


def test_gauss_matches_dense_nonseparable():
    """Pin 12: the per-axis passes equal the dense 3-D convolution with the isotropic Gaussian of
    the mm displacement (tests/brute.py), on a grid with unequal dimensions and voxel sizes."""
    rng = np.random.default_rng(32)
    dim, vs = (7, 6, 9), (1.65, 2.2, 2.0)
    x = rng.uniform(0, 1, size=dim)
    G = gauss_matrix(dim, vs, FWHM_RES)
    np.testing.assert_allclose(oracle.gauss3d(x, vs, FWHM_RES).ravel(), G @ x.ravel(), rtol=1e-12, atol=1e-15)


def test_gauss_delta_moments_fwhm():
    """Pin 13: a point source in the middle of a large grid spreads into a kernel of total weight 1
    whose second moment along every axis, in mm^2, is sigma^2 = (4.5 mm / 2.3548)^2 for any voxel
    size (the sampled, 4-sigma-truncated Gaussian differs from the continuous one by < 1e-3
    relative at sigma >= 1 voxel): the FWHM is the physical one, isotropic in mm."""
    vs = (1.0, 1.25, 1.5)
    dim = (41, 33, 29)
    x = np.zeros(dim)
    c = tuple(d // 2 for d in dim)
    x[c] = 1.0
    y = oracle.gauss3d(x, vs, FWHM_RES)
    assert y.sum() == pytest.approx(1.0, rel=1e-12)
    sig2 = (FWHM_RES / math.sqrt(8 * math.log(2))) ** 2
    for a in range(3):
        prof = y.sum(axis=tuple(b for b in range(3) if b != a))
        pos = (np.arange(dim[a]) - c[a]) * vs[a]
        assert np.sum(prof * pos) == pytest.approx(0.0, abs=1e-12)
        assert np.sum(prof * pos**2) == pytest.approx(sig2, rel=1e-3)


def test_gauss_self_adjoint_and_identity():
    """Pin 14: <G x, y> = <x, G y> (symmetric kernel, zero boundary: the operator is its own
    adjoint, which the OSEM back path relies on); FWHM 0 is the identity."""
    rng = np.random.default_rng(33)
    dim, vs = (12, 10, 8), (1.65, 1.65, 2.0)
    x, y = rng.standard_normal(dim), rng.standard_normal(dim)
    lhs = float(np.sum(oracle.gauss3d(x, vs, FWHM_RES) * y))
    rhs = float(np.sum(x * oracle.gauss3d(y, vs, FWHM_RES)))
    assert lhs == pytest.approx(rhs, rel=1e-12)
    np.testing.assert_array_equal(oracle.gauss3d(x, vs, 0.0), x)


def test_osem_resolution_model_dense_algebra():
    """Pin 15: OSEM with the resolution model equals the update written with dense matrices,
    system model A G (brute-force A, dense non-separable G): x <- x * G A_j^T (1 / (A_j G x + bg))
    / (sens / n_sub) with sens = G A_s^T 1 -- catches a blur applied on the wrong side, missing on
    the back path, or applied to the updated instead of the current image."""
    xs, xe, bins, dim, vs, origin, tof, _ = _osem_problem(seed=41)
    ss, se = random_rays(np.random.default_rng(42), 2000, origin, vs, dim)
    G = gauss_matrix(dim, vs, FWHM_RES)
    sens = (G @ oracle.back(ss, se, origin, vs, dim, np.ones(ss.shape[0])).ravel()).reshape(dim)
    A = system_matrix(xs, xe, origin, vs, dim, tof=tof, mode="lm", bins=bins)
    bg, n_iter, n_sub = 0.1, 2, 3
    s = sens.ravel()
    x = (s > 0).astype(float)
    for _ in range(n_iter):
        for j in range(n_sub):
            Aj = A[j::n_sub]
            ybar = Aj @ (G @ x) + bg
            acc = G.T @ (Aj.T @ (1.0 / ybar))
            x = np.where(s > 0, x * acc / np.where(s > 0, s / n_sub, 1.0), 0.0)
    got = oracle.lm_osem(xs, xe, bins, origin, vs, dim, tof, sens, bg, n_iter, n_sub, (sens > 0).astype(float),
                         fwhm=FWHM_RES)
    np.testing.assert_allclose(got.ravel(), x, rtol=1e-10, atol=1e-14)
    plain = oracle.lm_osem(xs, xe, bins, origin, vs, dim, tof, sens, bg, n_iter, n_sub, (sens > 0).astype(float))
    assert np.max(np.abs(plain - got)) > 1e-3 * np.max(got)  # the model matters on this problem
    zero = oracle.lm_osem(xs, xe, bins, origin, vs, dim, tof, sens, bg, n_iter, n_sub, (sens > 0).astype(float),
                          fwhm=0.0)
    np.testing.assert_array_equal(zero, plain)


# ------------------------------------------------ tabulated TOF kernel

def _skew_triangle(centre, left, right):
    """Asymmetric piecewise-linear kernel: 0 at centre - left, 1 at centre, 0 at centre + right."""

    def w(x):
        if centre - left < x <= centre:
            return (x - (centre - left)) / left
        if centre < x < centre + right:
            return ((centre + right) - x) / right
        return 0.0

    return w


def test_lut_kernel_matches_bruteforce():
    """Pin 16: a table whose nodes hold an asymmetric triangle kernel (breakpoints on nodes, so
    linear interpolation is exact) reproduces the brute-force system matrix built with the analytic
    kernel, for listmode and sinogram TOF, forward and back.  Catches a sign flip of the TOF
    coordinate, a wrong table origin or spacing, an index off by one."""
    rng = np.random.default_rng(71)
    dim, vs, origin = (6, 5, 4), (2.0, 2.5, 2.0), (-5.0, -5.0, -3.0)
    xs, xe = random_rays(rng, 40, origin, vs, dim)
    dx = 1.5
    centre, left, right = 3.0, 6.0, 12.0  # 4 and 8 steps of dx: node values k/4, k/8 exact in float32
    x0 = centre - left - 3 * dx
    nodes = x0 + dx * np.arange(int(round((centre + right + 2 * dx - x0) / dx)) + 1)
    w = _skew_triangle(centre, left, right)
    lut = np.array([w(x) for x in nodes], dtype=np.float32)
    tof = dict(tofd(4.0, 1.0, 3.0, 7), lut=lut, lut_x0=x0, lut_dx=dx)
    tof_b = dict(tofd(4.0, 1.0, 3.0, 7), weight_fn=w)
    bins = rng.integers(0, 7, size=40).astype(np.int16)
    img = rng.uniform(0, 1, size=dim)
    A = system_matrix(xs, xe, origin, vs, dim, tof=tof_b, mode="lm", bins=bins)
    np.testing.assert_allclose(oracle.fwd_tof_lm(xs, xe, origin, vs, dim, tof, bins, img), A @ img.ravel(),
                               rtol=1e-12, atol=1e-12)
    y = rng.uniform(0, 1, size=40)
    np.testing.assert_allclose(oracle.back_tof_lm(xs, xe, origin, vs, dim, tof, bins, y).ravel(), A.T @ y,
                               rtol=1e-12, atol=1e-12)
    As = system_matrix(xs, xe, origin, vs, dim, tof=tof_b, mode="sino")
    np.testing.assert_allclose(oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tof, img),
                               np.einsum("lbv,v->lb", As, img.ravel()), rtol=1e-12, atol=1e-12)
    assert np.abs(A).sum() > 0


def test_lut_gaussian_converges_quadratically():
    """Pin 17: tabulating the Gaussian bin weight (exact erf values, scipy) at spacing h and
    interpolating linearly reproduces the Gaussian projector with an error that falls as h^2
    (ratio ~4 per halving) and stays below h^2/8 * max|w''| relative to the largest weight."""
    rng = np.random.default_rng(72)
    dim, vs, origin = (12, 12, 6), (2.0, 2.0, 2.0), (-11.0, -11.0, -5.0)
    xs, xe = random_rays(rng, 200, origin, vs, dim)
    bw, sig, ns, nb = 8.0, 6.0, 3.0, 9
    tof = tofd(bw, sig, ns, nb)
    bins = rng.integers(0, nb, size=200).astype(np.int16)
    img = rng.uniform(0.5, 1.5, size=dim)
    exact = oracle.fwd_tof_lm(xs, xe, origin, vs, dim, tof, bins, img)

    def table(h):
        win = float(tof["n_sigmas"]) * float(tof["sigma"]) + 0.5 * float(tof["bin_width"])
        n = int(np.ceil(2 * win / h)) + 1
        x = -win + h * np.arange(n)
        tr = float(tof["n_sigmas"]) * float(tof["sigma"])
        G = lambda u: 0.5 * special.erf(np.clip(u, -tr, tr) / (np.sqrt(2) * float(tof["sigma"])))
        wv = G(x + 0.5 * float(tof["bin_width"])) - G(x - 0.5 * float(tof["bin_width"]))
        return dict(tof, lut=wv.astype(np.float32), lut_x0=-win, lut_dx=h), wv.max()

    errs = []
    for h in (0.4, 0.2, 0.1):
        t, wmax = table(h)
        got = oracle.fwd_tof_lm(xs, xe, origin, vs, dim, t, bins, img)
        errs.append(float(np.linalg.norm(got - exact) / np.linalg.norm(exact)))
        # max |w''| <= 2 max |g'| = 2 / (sigma^2 sqrt(2 pi e)) for the Gaussian density g
        bound = h * h / 8 * 2 / (sig**2 * np.sqrt(2 * np.pi * np.e)) / wmax
        assert errs[-1] <= bound
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, errs


def test_lut_adjoint_and_listmode_equals_sinogram():
    """Pin 18: with a tabulated kernel the listmode projector equals the sinogram projector's bin
    (bit-identical) and forward/back are adjoint to 1e-12."""
    rng = np.random.default_rng(73)
    dim, vs, origin = (8, 7, 5), (2.0, 2.0, 2.5), (-7.0, -6.0, -5.0)
    xs, xe = random_rays(rng, 60, origin, vs, dim)
    lut = np.abs(np.sin(np.linspace(0, 3.0, 37))).astype(np.float32)  # some non-Gaussian shape
    tof = dict(tofd(3.0, 1.0, 3.0, 5), lut=lut, lut_x0=-7.0, lut_dx=0.5)
    img = rng.uniform(0, 1, size=dim)
    sino = oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tof, img)
    for b in range(5):
        lm = oracle.fwd_tof_lm(xs, xe, origin, vs, dim, tof, np.full(60, b, np.int16), img)
        np.testing.assert_array_equal(lm, sino[:, b])
    y = rng.uniform(0, 1, size=(60, 5))
    lhs = float(np.sum(sino * y))
    rhs = float(np.sum(img * oracle.back_tof_sino(xs, xe, origin, vs, dim, tof, y)))
    assert lhs == pytest.approx(rhs, rel=1e-12)


# ------------------------------------- per-ray TOF parameters (generalising Sec. 2.2)

def _per_ray(rng, n, bad=True):
    """Per-ray sigma in [0.6, 2.5] mm and centre offset in [-3, 3] mm; with `bad`, a few entries
    that make their ray contribute nothing (sigma 0, negative, NaN; offset infinite)."""
    sig = rng.uniform(0.6, 2.5, size=n).astype(np.float32)
    off = rng.uniform(-3.0, 3.0, size=n).astype(np.float32)
    if bad:
        sig[3], sig[7], sig[11], off[15] = 0.0, -1.0, np.nan, np.inf
    return sig, off


@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_per_ray_tof_matches_bruteforce(gi):
    """Per-LOR TOF kernel width and centre offset: oracle == brute force whose rows use each
    ray's own sigma / offset in the quadrature weights; rays with an unusable entry give zero
    rows.  Catches the scalar sigma or offset leaking into a per-ray computation (in the erf
    scale, the truncation or the bin centre) and a per-ray array indexed by the wrong ray."""
    dim, vs, origin = GRIDS[gi]
    rng = np.random.default_rng(300 + gi)
    n = 30
    xs, xe = random_rays(rng, n, origin, vs, dim, inside_frac=0.2)
    sig, off = _per_ray(rng, n)
    for per in ({"sigma_per_ray": sig}, {"offset_per_ray": off}, {"sigma_per_ray": sig, "offset_per_ray": off}):
        tof = dict(tofd(bin_width=2.5, sigma=1.7, n_sigmas=2.5, n_bins=9, center_offset=0.4), **per)
        A = system_matrix(xs, xe, origin, vs, dim, tof=tof, mode="sino")
        x = rng.uniform(0, 1, size=dim)
        y = rng.uniform(0, 1, size=(n, tof["n_bins"]))
        fs = oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tof, x)
        np.testing.assert_allclose(fs, np.einsum("lbv,v->lb", A, x.ravel()), rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(oracle.back_tof_sino(xs, xe, origin, vs, dim, tof, y).ravel(),
                                   np.einsum("lbv,lb->v", A, y), rtol=1e-11, atol=1e-12)
        bins = rng.integers(0, tof["n_bins"], size=n).astype(np.int16)
        Alm = system_matrix(xs, xe, origin, vs, dim, tof=tof, mode="lm", bins=bins)
        ylm = rng.uniform(0, 1, size=n)
        fl = oracle.fwd_tof_lm(xs, xe, origin, vs, dim, tof, bins, x)
        np.testing.assert_allclose(fl, Alm @ x.ravel(), rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(oracle.back_tof_lm(xs, xe, origin, vs, dim, tof, bins, ylm).ravel(),
                                   Alm.T @ ylm, rtol=1e-11, atol=1e-12)
        dead = [3, 7, 11] if "sigma_per_ray" in per else []
        dead += [15] if "offset_per_ray" in per else []
        assert not np.any(fs[dead]) and not np.any(fl[dead])
        assert np.count_nonzero(fs.sum(1)) > 10


def test_per_ray_tof_work_counter():
    """The work counter with per-ray sigma / offset: a sample counts iff its stencil touches the
    grid and it lies strictly inside the bin's support |s - c_b| < n_sigmas sigma_l + bw / 2
    (written out per plane here, centre from the ray's own offset)."""
    dim, vs, origin = GRIDS[0]
    rng = np.random.default_rng(17)
    n = 40
    xs, xe = random_rays(rng, n, origin, vs, dim, inside_frac=0.2)
    sig, off = _per_ray(rng, n)
    tof = dict(tofd(bin_width=2.0, sigma=1.0, n_sigmas=2.5, n_bins=7), sigma_per_ray=sig, offset_per_ray=off)
    bins = rng.integers(0, 7, size=n).astype(np.int16)
    tot, per = oracle.count_samples(xs, xe, origin, vs, dim, tof=tof, bins=bins, per_ray=True)
    for l in range(n):
        s_l, o_l = float(sig[l]), float(off[l])
        usable = math.isfinite(s_l) and s_l > 0 and math.isfinite(o_l)
        d32 = (xe[l] - xs[l]).astype(np.float32)
        p = int(np.argmax(np.abs(d32)))
        inplane = [a for a in range(3) if a != p]
        a64, b64 = xs[l].astype(float), xe[l].astype(float)
        length = float(np.linalg.norm(b64 - a64))
        cb = (int(bins[l]) - 3) * float(tof["bin_width"]) + o_l if usable else 0.0
        cnt = 0
        for k in range(dim[p]):
            t = (origin[p] + k * vs[p] - a64[p]) / (b64[p] - a64[p])
            if not usable or t < 0 or t > 1:
                continue
            X = a64 + t * (b64 - a64)
            idx = [(X[a] - origin[a]) / vs[a] for a in inplane]
            touch = all(math.floor(i) + 1 >= 0 and math.floor(i) <= dim[a] - 1 for i, a in zip(idx, inplane))
            inside = abs((t - 0.5) * length - cb) < float(tof["n_sigmas"]) * s_l + 0.5 * float(tof["bin_width"])
            cnt += touch and inside
        assert per[l] == cnt, l
    assert tot == per.sum() > 0


def test_per_ray_offset_shifts_bins():
    """A per-ray centre offset of k bin widths moves every bin centre of that ray by k bins
    towards the end point: column t with offset k * bw equals column t + k without offset.
    Catches a sign error of the offset, or an offset applied to the sample instead of the bin."""
    rng = np.random.default_rng(18)
    dim, vs, origin = (20, 18, 8), (2.0, 2.0, 2.0), (-19.0, -17.0, -7.0)
    n, nb, bw = 40, 41, 4.0
    xs, xe = random_rays(rng, n, origin, vs, dim)
    x = rng.uniform(size=dim)
    k = rng.integers(-3, 4, size=n)
    tof0 = tofd(bw, 3.0, 3.0, nb)
    ref = oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tof0, x)
    sh = oracle.fwd_tof_sino(xs, xe, origin, vs, dim, dict(tof0, offset_per_ray=(k * bw).astype(np.float32)), x)
    for l in range(n):
        t = np.arange(max(0, -k[l]), min(nb, nb - k[l]))
        np.testing.assert_allclose(sh[l, t], ref[l, t + k[l]], rtol=1e-12, atol=1e-15)
    assert np.any(k != 0) and np.count_nonzero(ref) > 0


def test_per_ray_sigma_bin_sum_and_adjoint():
    """With each ray's own sigma the TOF weights of a fully covered LOR still telescope to
    erf(n_sigmas / sqrt 2) times the non-TOF projection (the mass of the truncated Gaussian does
    not depend on its width), and the per-ray back projection is the exact adjoint.  Catches a
    truncation or an erf scale that mixes the scalar and the per-ray sigma."""
    rng = np.random.default_rng(19)
    dim, vs, origin = (20, 18, 8), (2.0, 2.0, 2.0), (-19.0, -17.0, -7.0)
    n = 50
    xs, xe = random_rays(rng, n, origin, vs, dim)
    x = rng.uniform(size=dim)
    sig = rng.uniform(1.0, 6.0, size=n).astype(np.float32)
    tof = dict(tofd(4.0, 3.0, 3.0, 41), sigma_per_ray=sig)  # bins cover +-82 mm
    pt = oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tof, x)
    pn = oracle.fwd(xs, xe, origin, vs, dim, x)
    np.testing.assert_allclose(pt.sum(1), special.erf(3.0 / math.sqrt(2.0)) * pn, rtol=1e-13, atol=1e-13)
    y = rng.uniform(size=(n, 41))
    lhs = float(np.sum(pt * y))
    rhs = float(np.sum(x * oracle.back_tof_sino(xs, xe, origin, vs, dim, tof, y)))
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # arrays holding the scalar values reproduce the scalar path exactly
    same = dict(tofd(4.0, 3.0, 3.0, 41, center_offset=1.5), sigma_per_ray=np.full(n, 3.0, np.float32),
                offset_per_ray=np.full(n, 1.5, np.float32))
    assert np.array_equal(oracle.fwd_tof_sino(xs, xe, origin, vs, dim, same, x),
                          oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tofd(4.0, 3.0, 3.0, 41, 1.5), x))


def test_lut_work_counter():
    """The work counter with a tabulated kernel: a sample counts iff its stencil touches the grid
    and its signed distance x from the event's bin centre lies strictly inside the table's range
    (x0, x0 + (n - 1) dx) -- also with a per-ray centre offset (written out per plane here, the
    bin centre from the ray's own offset).  The table values play no part (a zero entry still
    counts).  Catches a closed range, a table origin taken from the wrong side of the bin centre,
    or an offset ignored in the count."""
    dim, vs, origin = GRIDS[0]
    rng = np.random.default_rng(19)
    n = 60
    xs, xe = random_rays(rng, n, origin, vs, dim, inside_frac=0.2)
    x0, dx, n_lut = -3.7, 0.45, 15  # asymmetric: (x0, x0 + 14 dx) = (-3.7, 2.6)
    lut = np.zeros(n_lut, dtype=np.float32)
    lut[3:9] = 1.0
    bins = rng.integers(-1, 8, size=n).astype(np.int16)  # -1 and 7: outside the 7 bins
    for with_offset in (False, True):
        off = rng.normal(0.0, 1.5, size=n).astype(np.float32) if with_offset else None
        tof = dict(tofd(bin_width=2.0, sigma=1.0, n_sigmas=2.5, n_bins=7), lut=lut, lut_x0=x0, lut_dx=dx)
        if with_offset:
            tof["offset_per_ray"] = off
        tot, per = oracle.count_samples(xs, xe, origin, vs, dim, tof=tof, bins=bins, per_ray=True)
        lo, hi = x0, x0 + (n_lut - 1) * dx
        for l in range(n):
            d32 = (xe[l] - xs[l]).astype(np.float32)
            p = int(np.argmax(np.abs(d32)))
            inplane = [a for a in range(3) if a != p]
            a64, b64 = xs[l].astype(float), xe[l].astype(float)
            length = float(np.linalg.norm(b64 - a64))
            b = int(bins[l])
            cnt = 0
            if 0 <= b < 7:
                cb = (b - 3) * 2.0 + (float(off[l]) if with_offset else 0.0)
                for k in range(dim[p]):
                    t = (origin[p] + k * vs[p] - a64[p]) / (b64[p] - a64[p])
                    if t < 0 or t > 1:
                        continue
                    X = a64 + t * (b64 - a64)
                    idx = [(X[a] - origin[a]) / vs[a] for a in inplane]
                    touch = all(math.floor(i) + 1 >= 0 and math.floor(i) <= dim[a] - 1 for i, a in zip(idx, inplane))
                    x = (t - 0.5) * length - cb
                    cnt += touch and lo < x < hi
            assert per[l] == cnt, (with_offset, l)
        assert tot == per.sum() > 0


def test_tof_kernel_values_textbook():
    """The oracle's TOF bin weight w(x) (bin centre at x = 0) equals the truncated-normal mass
    over the bin: Phi(min(x + bw/2, T)/sigma) - Phi(max(x - bw/2, -T)/sigma), T = n_sigmas sigma,
    and 0 once the bin lies beyond the truncation (scipy's normal CDF, not erf).  Catches a
    truncation applied after the convolution, a missing 1/2 or sqrt(2)."""
    bw, sig, ns = 28.0, 58.5 / 2.355, 3.0
    t = tofd(bw, sig, ns, 1)
    x = np.linspace(-120.0, 120.0, 2401)
    w = oracle.tof_kernel(x, t)
    s, T = float(t["sigma"]), float(t["n_sigmas"]) * float(t["sigma"])
    hb = 0.5 * float(t["bin_width"])
    a = np.clip(x - hb, -T, T)
    b = np.clip(x + hb, -T, T)
    ref = stats.norm.cdf(b / s) - stats.norm.cdf(a / s)
    np.testing.assert_allclose(w, ref, rtol=0, atol=2e-15)
    assert np.all(w[np.abs(x) >= T + hb] == 0.0) and w.max() > 0.4


# --------------------------------------------------- TOF sinogram OSEM

def _sino_osem_problem(seed=31, n=90):
    rng = np.random.default_rng(seed)
    dim, vs, origin = (6, 5, 4), (2.0, 2.5, 2.0), (-5.0, -5.0, -3.0)
    xs, xe = random_rays(rng, n, origin, vs, dim)
    tof = tofd(3.0, 2.0, 3.0, 7)
    sub = rng.integers(0, 3, size=n).astype(np.int32)
    sub[::17] = -1  # LORs in no subset
    y = rng.poisson(2.0, size=(n, 7)).astype(np.float64)
    return rng, xs, xe, dim, vs, origin, tof, sub, y


def test_tof_sino_osem_matches_dense_algebra():
    """TOF sinogram OSEM equals the same update written with the brute-force TOF matrix
    (quadrature weights, tent functions) and numpy algebra: per subset j (LORs with sub == j),
    x <- x * A_j^T (y / (A_j x + bg)) / A_j^T 1, zero where A_j^T 1 == 0.  Catches a subset taken
    from the wrong LORs, a sensitivity of all subsets, the ratio inverted, or the background
    dropped."""
    rng, xs, xe, dim, vs, origin, tof, sub, y = _sino_osem_problem()
    A = system_matrix(xs, xe, origin, vs, dim, tof=tof, mode="sino")  # [n, nb, nv]
    bg, n_iter = 0.3, 2
    x = rng.uniform(0.5, 1.5, size=dim)
    ref = x.ravel().copy()
    for _ in range(n_iter):
        for j in range(3):
            Aj = A[sub == j].reshape(-1, A.shape[2])
            yj = y[sub == j].ravel()
            sens = Aj.sum(axis=0)
            e = Aj @ ref + bg
            acc = Aj.T @ np.where(e > 0, yj / np.where(e > 0, e, 1.0), 0.0)
            ref = np.where(sens > 0, ref * acc / np.where(sens > 0, sens, 1.0), 0.0)
    got = oracle.tof_sino_osem(xs, xe, sub, 3, origin, vs, dim, tof, y, bg, n_iter, x)
    np.testing.assert_allclose(got.ravel(), ref, rtol=1e-11, atol=1e-14)
    assert np.count_nonzero(ref == 0) > 0 and np.count_nonzero(ref > 0) > 60


def test_tof_sino_osem_count_conservation():
    """With zero background, one subset update satisfies sum_v sens_j,v x_v^new = sum of the
    subset's counts over (LOR, bin) pairs with positive expectation (exact EM invariant)."""
    rng, xs, xe, dim, vs, origin, tof, sub, y = _sino_osem_problem(seed=32, n=120)
    one_sub = np.where(sub >= 0, 0, -1).astype(np.int32)
    x0 = rng.uniform(0.5, 2.0, size=dim)
    x1 = oracle.tof_sino_osem(xs, xe, one_sub, 1, origin, vs, dim, tof, y, 0.0, 1, x0)
    m = one_sub == 0
    sens = oracle.back_tof_sino(xs[m], xe[m], origin, vs, dim, tof, np.ones((int(m.sum()), 7)))
    ybar = oracle.fwd_tof_sino(xs[m], xe[m], origin, vs, dim, tof, x0)
    counts = float(y[m][ybar > 0].sum())
    assert counts > 100
    assert float(np.sum(sens * x1)) == pytest.approx(counts, rel=1e-12)
