"""Pins of the oracle's background subtraction (Background Subtraction
section and its figure: sources outside a sink group's neighbourhood become
matter minus the uniform mean density, the uniform cube of each multipole
cell subtracted to the order of its matter expansion, the neighbourhood's and
the leftover regions' background removed through the exact field of a
uniform box).

Checked against the mathematics, not against the oracle's own formulas: the
box field against Gauss-Legendre quadrature of its defining volume integral,
Gauss's law, the interior of a cube (zero at the centre, the isotropic linear
law -4 pi rho u / 3 near it), the far field of a cube (a point mass up to a
relative (s/d)^4 term, its first non-vanishing multipole being the fourth);
the cube moments through the convergence of their truncated expansion to
that exact field; the bookkeeping of the lists through a tiling of the near
zone (every point of the 5L cube covered exactly once by the subtracted
pieces and the neighbourhood) and through the identity that ties the
subtracted result to the unsubtracted one (they differ only by the
truncation of the subtracted cubes); the purpose of the method: in a
perfect lattice, whose exact periodic force is zero, and in a perturbed one,
the subtracted treecode is more accurate at the same order; and the VJP
(the box field's gradient against differences and Poisson's equation, the
whole VJP against differences in positions and masses)."""
import numpy as np
import pytest

BOX = np.array([0.0, 0.0, 0.0, 1.0])


def _lattice(n1, amp, seed):
    g = (np.arange(n1) + 0.5) / n1
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    x = (x + amp / n1 * np.random.default_rng(seed).standard_normal(x.shape)) % 1.0
    return x, np.full(x.shape[0], 1.0 / x.shape[0])


def _quad_field(lo, hi, x, ng=48):
    """The defining integral of the box field by tensor Gauss-Legendre."""
    gx, gw = np.polynomial.legendre.leggauss(ng)
    ys = [0.5 * (hi[d] - lo[d]) * gx + 0.5 * (hi[d] + lo[d]) for d in range(3)]
    ws = [0.5 * (hi[d] - lo[d]) * gw for d in range(3)]
    y = np.stack(np.meshgrid(*ys, indexing="ij"), -1).reshape(-1, 3)
    w = np.einsum("i,j,k->ijk", *ws).reshape(-1)
    r = y - x
    d = np.linalg.norm(r, axis=1)
    return (w[:, None] * r / d[:, None] ** 3).sum(0)


def test_box_field_vs_quadrature(orc):
    lo, hi = np.array([0.1, -0.2, 0.3]), np.array([0.6, 0.5, 0.45])
    pts = np.array([[1.2, 0.7, -0.4], [-0.5, 0.15, 0.375], [0.35, -0.9, 0.4], [0.35, 0.15, 1.0],
                    [0.6, 0.5, 0.75]])  # the last one level with a corner's x and y
    a = orc.box_field(lo, hi, pts)
    for x, ax in zip(pts, a):
        q = _quad_field(lo, hi, x)
        assert np.linalg.norm(ax - q) <= 1e-10 * np.linalg.norm(q)


def test_box_field_gauss_law(orc):
    lo, hi = np.array([-0.3, -0.1, -0.25]), np.array([0.2, 0.35, 0.1])
    vol = np.prod(hi - lo)
    ct, wt = np.polynomial.legendre.leggauss(40)
    ph = (np.arange(80) + 0.5) * 2 * np.pi / 80
    st = np.sqrt(1 - ct ** 2)
    n = np.stack([st[:, None] * np.cos(ph)[None, :], st[:, None] * np.sin(ph)[None, :],
                  np.broadcast_to(ct[:, None], (40, 80))], -1).reshape(-1, 3)
    w = (wt[:, None] * np.full(80, 2 * np.pi / 80)[None, :]).reshape(-1)
    for centre, R, enclosed in (((0.0, 0.0, 0.0), 1.0, True), ((2.0, 0.5, -1.0), 0.8, False)):
        x = np.array(centre) + R * n
        a = orc.box_field(lo, hi, x)
        flux = R * R * np.sum(w * np.einsum("ij,ij->i", a, n))
        want = -4 * np.pi * vol if enclosed else 0.0
        assert abs(flux - want) <= 1e-8 * 4 * np.pi * vol


def test_box_field_cube_interior(orc):
    lo, hi = np.zeros(3), np.ones(3)
    assert np.abs(orc.box_field(lo, hi, [0.5, 0.5, 0.5])).max() <= 1e-14
    u = np.array([1e-3, -2e-3, 0.5e-3])
    a = orc.box_field(lo, hi, 0.5 + u)[0]
    lin = -4 * np.pi / 3 * u
    # the next term is cubic in u (the potential's quartic cubic harmonic)
    assert np.linalg.norm(a - lin) <= 1e-4 * np.linalg.norm(lin)
    # cubic symmetry: a permutation of the offset permutes the field
    b = orc.box_field(lo, hi, 0.5 + u[[2, 0, 1]])[0]
    assert np.allclose(b, a[[2, 0, 1]], rtol=1e-12, atol=0)


def test_box_field_cube_far_field(orc):
    s = 0.25
    lo, hi = np.full(3, -s / 2), np.full(3, s / 2)
    dirn = np.array([0.6, -0.48, 0.64])
    errs = []
    for d in (8 * s, 16 * s):
        x = d * dirn
        a = orc.box_field(lo, hi, x)[0]
        pm = -s ** 3 * x / d ** 3
        errs.append(np.linalg.norm(a - pm) / np.linalg.norm(pm))
    assert errs[1] <= 1e-4
    assert 14.0 <= errs[0] / errs[1] <= 18.0  # (s/d)^4


def test_cube_moments_expansion_converges_to_exact(orc):
    """The truncated expansion of a uniform cube (its moments, unit density)
    approaches the exact box field with the order, even orders only."""
    s = 0.5
    lo, hi = np.full(3, -s / 2), np.full(3, s / 2)
    x = np.array([0.9, 0.55, -0.7])
    exact = orc.box_field(lo, hi, x)[0]
    errs = []
    for p in (0, 2, 4, 6, 8):
        a, _ = orc.m2p(p, orc.cube_moments(p, s), x, 0.0)
        errs.append(np.linalg.norm(a - exact) / np.linalg.norm(exact))
    # a cube's quadrupole is isotropic: it adds no field
    assert abs(errs[1] - errs[0]) <= 1e-12
    assert errs[0] > errs[2] > errs[3] > errs[4]
    assert errs[-1] <= 1e-6
    M = orc.cube_moments(3, s)
    assert M[0] == s ** 3
    # order 2: s^5 / 12 on the diagonal, nothing off it
    assert np.isclose(M[4], s ** 5 / 12, rtol=1e-15) and M[5] == 0.0


def _bs_tree(orc, pos, mass, theta, n_leaf, n_group, p=None):
    t = orc.Tree(pos, n_leaf, n_group, BOX)
    t.build_lists_periodic_bs(theta, 0)
    if p is not None:
        t.compute_moments(pos, mass, p)
    return t


def _neigh(cells, gc, width):
    h = 0.5 ** (int(cells["level"][gc]) + 1)
    c = cells["centre"][gc]
    return c - width * h, c + width * h


def _clustered(n, width, seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.random((n // 2, 3)),
                        (0.3 + width * rng.standard_normal((n - n // 2, 3))) % 1.0])
    return x, np.full(n, 1.0 / n)


@pytest.mark.parametrize("kind,n,a,n_leaf,n_group,width", [
    ("lattice", 12, 0.2, 8, 32, 3), ("lattice", 16, 0.6, 16, 64, 3),
    ("clustered", 3000, 0.04, 8, 32, 3),  # coarse leaves straddle fine neighbourhoods
    ("clustered", 3000, 0.1, 16, 64, 5),
])
def test_bs_pieces_tile_the_near_zone(orc, kind, n, a, n_leaf, n_group, width):
    pos, mass = _lattice(n, a, 5) if kind == "lattice" else _clustered(n, a, 11)
    t = orc.Tree(pos, n_leaf, n_group, BOX)
    t.build_lists_periodic_bs(0.6, 0, width=width)
    cells, groups = t.cells(), t.groups()
    po, pl, mo, ml = t.lists()
    pi, mi = t.list_images()
    off, boxes, sign, sub = t.background()
    lev = cells["level"]
    rng = np.random.default_rng(6)
    assert sub.sum() > 0
    if kind == "clustered":
        assert (sign > 0).sum() > 0 and (sign < 0).sum() > 0
    for g in range(len(groups)):
        # signed volume: subtracted cubes + boxes + N(g) = the 5L cube, exactly
        vol = sum(0.5 ** (3 * int(lev[ml[e]])) for e in range(mo[g], mo[g + 1]) if sub[e])
        bx = boxes[off[g]:off[g + 1]]
        vol += float((-sign[off[g]:off[g + 1]] * np.prod(bx[:, 3:] - bx[:, :3], axis=1)).sum())
        vol += (width * 0.5 ** int(lev[groups[g]])) ** 3
        assert vol == 125.0
        if g % 7:
            continue
        # coverage: random points of the 5L cube are covered exactly once
        nlo, nhi = _neigh(cells, groups[g], width)
        pieces = [(cells["centre"][ml[e]] + _shift(mi[e]) - 0.5 ** (lev[ml[e]] + 1),
                   cells["centre"][ml[e]] + _shift(mi[e]) + 0.5 ** (lev[ml[e]] + 1), -1)
                  for e in range(mo[g], mo[g + 1]) if sub[e]]
        pieces += [(b[:3], b[3:], int(sg)) for b, sg in zip(bx, sign[off[g]:off[g + 1]])]
        pieces.append((nlo, nhi, -1))
        y = rng.random((400, 3)) * 5.0 - 2.0
        cover = np.zeros(len(y))
        for lo, hi, sg in pieces:
            inside = np.all((y > lo) & (y < hi), axis=1)
            cover -= sg * inside
        assert np.all(cover == 1)
        # no M2P entry straddles N(g); the flag says which side it is on
        for e in range(mo[g], mo[g + 1]):
            c = ml[e]
            h = 0.5 ** (lev[c] + 1)
            lo, hi = cells["centre"][c] + _shift(mi[e]) - h, cells["centre"][c] + _shift(mi[e]) + h
            inside = np.all(lo >= nlo) and np.all(hi <= nhi)
            outside = np.any(hi <= nlo) or np.any(lo >= nhi)
            assert inside or outside
            assert bool(sub[e]) == outside


def _shift(img):
    img = int(img)
    return np.array([img // 25 - 2, (img // 5) % 5 - 2, img % 5 - 2], dtype=np.float64)


def test_bs_differs_from_plain_only_by_cube_truncation(orc):
    """Subtracted minus unsubtracted forces = rho times the sum over the
    subtracted M2P cells of (exact cube field - its order-p expansion): every
    other background piece cancels exactly. Lists are the same when no cell
    straddles a neighbourhood (checked)."""
    pos, mass = _lattice(12, 0.3, 8)
    eps, p, theta = 1e-3, 4, 0.5
    tb = _bs_tree(orc, pos, mass, theta, 8, 32, p)
    tp = orc.Tree(pos, 8, 32, BOX)
    tp.build_lists_periodic(theta, 0)
    tp.compute_moments(pos, mass, p)
    if not all(np.array_equal(a, b) for a, b in zip(tb.lists(), tp.lists())):
        pytest.skip("a straddling cell changed the lists")
    sinks = np.sort(np.random.default_rng(9).choice(pos.shape[0], 24, replace=False))
    ab, _, _ = tb.eval(pos, mass, eps, sinks=sinks, with_pot=False)
    ap, _, _ = tp.eval(pos, mass, eps, sinks=sinks, with_pot=False)
    cells = tb.cells()
    po, pl, mo, ml = tb.lists()
    _, mi = tb.list_images()
    _, _, _, sub = tb.background()
    grp = tb.group_of()[np.argsort(tb.keys()[1])]
    rho = mass.sum()
    for k, i in enumerate(sinks):
        g = grp[i]
        want = np.zeros(3)
        for e in range(mo[g], mo[g + 1]):
            if not sub[e]:
                continue
            c = ml[e]
            s = 0.5 ** int(cells["level"][c])
            cc = cells["centre"][c] + _shift(mi[e])
            exact = orc.box_field(cc - s / 2, cc + s / 2, pos[i])[0]
            trunc, _ = orc.m2p(p, orc.cube_moments(p, s), pos[i] - cc, eps)
            want += rho * (exact - trunc)
        assert np.linalg.norm((ab[k] - ap[k]) - want) <= 1e-11


def test_bs_more_accurate_in_lattices(orc):
    eps, p = 1e-3, 6
    # perfect lattice: the exact periodic force vanishes at every particle
    pos, mass = _lattice(16, 0.0, 0)
    sinks = np.sort(np.random.default_rng(1).choice(pos.shape[0], 48, replace=False))
    res = {}
    for bs in (False, True):
        t = orc.Tree(pos, 16, 64, BOX)
        (t.build_lists_periodic_bs if bs else t.build_lists_periodic)(0.6, 0)
        t.compute_moments(pos, mass, p)
        res[bs] = np.sqrt((t.eval(pos, mass, eps, sinks=sinks, with_pot=False)[0] ** 2).sum(1).mean())
    assert res[True] <= res[False] / 5
    # perturbed lattice against the Ewald direct sum
    pos, mass = _lattice(16, 0.05, 3)
    ad = orc.ewald_direct(pos, mass, 1.0, eps, sinks=sinks)
    for bs in (False, True):
        t = orc.Tree(pos, 8, 32, BOX)
        (t.build_lists_periodic_bs if bs else t.build_lists_periodic)(0.6, 0)
        t.compute_moments(pos, mass, p)
        a = t.eval(pos, mass, eps, sinks=sinks, with_pot=False)[0]
        res[bs] = np.sqrt(((a - ad) ** 2).sum(1).mean())
    assert res[True] <= res[False] / 1.5


def test_box_grad_against_differences_and_poisson(orc):
    """The gradient of the box field against central differences of the
    field, and its trace: -4 pi inside the box, 0 outside (Poisson)."""
    lo, hi = np.array([0.1, -0.2, 0.3]), np.array([0.6, 0.5, 0.45])
    pts = np.array([[1.2, 0.7, -0.4], [0.35, 0.15, 0.375], [0.35, 0.15, 1.0], [0.6, 0.1, 0.2],
                    [0.2, -0.1, 0.32]])
    T = orc.box_grad(lo, hi, pts)
    h = 1e-5
    for x, Tx in zip(pts, T):
        F = np.stack([(orc.box_field(lo, hi, x + h * e)[0] - orc.box_field(lo, hi, x - h * e)[0])
                      / (2 * h) for e in np.eye(3)], axis=1)
        assert np.abs(Tx - F).max() <= 1e-7 * np.abs(F).max()
        assert np.allclose(Tx, Tx.T, rtol=0, atol=1e-14)
        inside = np.all((x > lo) & (x < hi))
        assert abs(np.trace(Tx) - (-4 * np.pi if inside else 0.0)) <= 1e-12


@pytest.mark.parametrize("kind", ["lattice", "clustered"])
def test_bs_vjp_matches_fd(orc, kind):
    """The VJP of background-subtracted lists (subtracted moments at the sink,
    the exact box fields and their gradients, the mean density through every
    mass) against Richardson-extrapolated central differences of the
    evaluation on the same lists, in positions and in masses."""
    if kind == "lattice":
        pos, mass = _lattice(10, 0.3, 12)
        t = orc.Tree(pos, 8, 32, BOX)
        t.build_lists_periodic_bs(0.5, 0, width=3)
    else:
        pos, mass = _clustered(1200, 0.04, 13)
        mass = mass * (0.5 + np.random.default_rng(14).random(mass.shape))
        t = orc.Tree(pos, 8, 32, BOX)
        t.build_lists_periodic_bs(0.6, 4, width=3)
        assert (t.background()[2] > 0).any()
    p, eps = 4, 1e-2
    t.compute_moments(pos, mass, p)
    abar = W_cot(pos.shape[0], 15)
    xb, mb = t.vjp(pos, mass, eps, abar)

    def L(x, m):
        t.compute_moments(x, m, p)
        a, _, _ = t.eval(x, m, eps, with_pot=False)
        return float((a * abar).sum())

    rng = np.random.default_rng(16)
    v, dm = rng.normal(size=pos.shape), rng.normal(size=mass.shape) * mass
    h = 1e-6

    def cd(fx, hh):
        return (fx(hh) - fx(-hh)) / (2 * hh)

    fx = lambda hh: L(pos + hh * v, mass)
    fm = lambda hh: L(pos, mass + hh * dm)
    fd_x = (4 * cd(fx, h) - cd(fx, 2 * h)) / 3
    fd_m = (4 * cd(fm, h) - cd(fm, 2 * h)) / 3
    assert abs(float((xb * v).sum()) - fd_x) <= 1e-7 * abs(fd_x)
    assert abs(float((mb * dm).sum()) - fd_m) <= 1e-7 * abs(fd_m)


def W_cot(n, seed):
    a = np.random.default_rng(seed).standard_normal((n, 3))
    return a / np.linalg.norm(a)


def test_bs_refusals(orc):
    pos, mass = _lattice(8, 0.2, 1)
    t = _bs_tree(orc, pos, mass, 0.5, 8, 32, 4)
    t.build_lists_periodic(0.5, 0)
    with pytest.raises(RuntimeError):
        t.background()
