"""Direct pins of the oracle's multigrid transfers (Appendix C), level 0 to
level 1, each one read back from unit vectors or checked on fields whose
transfer is known exactly:

  - face restriction: the printed 6-point stencil in 2D (weights 1/8 on the
    four faces offset along the normal, 1/4 on the two coincident faces) and
    its 12-point tensor extension in 3D (1/16 on eight offset faces, 1/8 on
    four coincident faces; a reading, the paper prints 2D only);
  - face prolongation: the printed 2D cases (3/4, 1/4 along the tangent;
    3/8, 1/8 for fine faces between coarse faces) and their mirror images
    for odd tangential index (a reading, the paper prints only even j);
  - at a wall the missing coarse tangential neighbour is the odd reflection
    (no-slip: the fine row next to the wall takes 1/2 of its coarse value,
    consistent with zero velocity on the wall) or the even reflection
    (free-slip: weight 1, consistent with zero normal derivative);
  - restriction and prolongation reproduce linear fields exactly wherever
    their stencil stays inside the grid, a property that does not depend on
    how the weights are written down, and the wall rules reproduce a field
    that vanishes on a no-slip wall (odd) and a constant across a free-slip
    wall (even);
  - cell restriction is the mean of the 2^d fine cells and cell prolongation
    injection.
A wrong weight, a wrong offset or a wrong reflection sign in any of the four
transfer functions fails at least one of these."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1308_4605_amd import workloads as W


def _ctx(dim, n, bc):
    lay = W.make_layout(dim, n, bc)
    rho, mu = W.random_coefficients(91, lay)
    o = oracle.Oracle(dim, lay.n, lay.bc, 1.0 / lay.n[0], 2.0, rho, mu)
    coarse = W.make_layout(dim, tuple(x // 2 for x in lay.n[:dim]) + (1,) * (3 - dim), bc)
    assert o.level_sizes(1) == (coarse.nvel, coarse.ncell)
    return o, lay, coarse


def _faces(lay):
    """(k, face index (i0, i1, i2), flat position) of every stored face."""
    out = []
    for k in range(lay.dim):
        dm = lay.face_dims(k)
        for i2 in range(dm[2] if lay.dim == 3 else 1):
            for i1 in range(dm[1]):
                for i0 in range(dm[0]):
                    q = lay.face_offsets[k] + i0 + dm[0] * (i1 + dm[1] * i2)
                    out.append((k, (i0, i1, i2), q))
    return out


def _is_wall(lay, k, f):
    return lay.wall(k) and f[k] in (0, lay.n[k])


def _pos(lay, k, f):
    """Flat position of face f of component k, periodic indices wrapped;
    None outside a walled axis."""
    dm = lay.face_dims(k)
    g = list(f)
    for a in range(lay.dim):
        if lay.wall(a):
            if not (0 <= g[a] < dm[a]):
                return None
        else:
            g[a] %= lay.n[a]
    return lay.face_offsets[k] + g[0] + dm[0] * (g[1] + dm[1] * g[2])


def _matrix(apply, n_in, n_out):
    M = np.zeros((n_out, n_in))
    e = np.zeros(n_in)
    for j in range(n_in):
        e[:] = 0.0
        e[j] = 1.0
        M[:, j] = apply(e)
    return M


def _centre(k, f, h):
    return np.array([f[a] * h if a == k else (f[a] + 0.5) * h for a in range(3)])


# ---------------------------------------------------------------- restriction

GRIDS_2D = [(8, 8), (8, 4)]
BCS_2D = [(0, 0), (1, 1), (2, 0), (3, 4)]


@pytest.mark.parametrize("n", GRIDS_2D)
@pytest.mark.parametrize("bc", BCS_2D)
def test_face_restriction_2d_is_the_printed_six_point_stencil(n, bc):
    o, lay, cl = _ctx(2, n, bc)
    R = _matrix(lambda v: o.restrict_faces(0, v), lay.nvel, cl.nvel)
    expect = np.zeros_like(R)
    for k, F, qc in _faces(cl):
        if _is_wall(cl, k, F):
            continue
        t = 1 - k  # tangential axis
        # the printed x-face formula, with the roles of the axes swapped for
        # y-faces: 1/8 at normal offsets -1, +1 and 1/4 at offset 0, over the
        # two fine rows 2J, 2J+1 along the tangent
        for off, wgt in ((-1, 1 / 8), (0, 1 / 4), (1, 1 / 8)):
            for row in (0, 1):
                f = [0, 0, 0]
                f[k] = 2 * F[k] + off
                f[t] = 2 * F[t] + row
                if _is_wall(lay, k, f):
                    continue  # wall faces carry no unknown
                q = _pos(lay, k, f)
                assert q is not None
                expect[qc, q] += wgt
    assert np.array_equal(R, expect)


@pytest.mark.parametrize("n,bc", [((4, 4, 4), (0, 0, 0)), ((8, 4, 4), (1, 0, 2)),
                                  ((4, 8, 4), (3, 1, 4))])
def test_face_restriction_3d_is_the_twelve_point_tensor_stencil(n, bc):
    o, lay, cl = _ctx(3, n, bc)
    R = _matrix(lambda v: o.restrict_faces(0, v), lay.nvel, cl.nvel)
    expect = np.zeros_like(R)
    for k, F, qc in _faces(cl):
        if _is_wall(cl, k, F):
            continue
        t1, t2 = [a for a in range(3) if a != k]
        # 1/8 on the four coincident faces, 1/16 on the eight offset ones
        for off, wgt in ((-1, 1 / 16), (0, 1 / 8), (1, 1 / 16)):
            for r1, r2 in itertools.product((0, 1), (0, 1)):
                f = [0, 0, 0]
                f[k], f[t1], f[t2] = 2 * F[k] + off, 2 * F[t1] + r1, 2 * F[t2] + r2
                if _is_wall(lay, k, f):
                    continue
                expect[qc, _pos(lay, k, f)] += wgt
    assert np.array_equal(R, expect)
    # each interior coarse face sums its twelve weights to one
    rows = [qc for k, F, qc in _faces(cl) if not _is_wall(cl, k, F)
            and not (lay.wall(k) and F[k] in (1, cl.n[k] - 1))]
    assert np.allclose(R[rows].sum(axis=1), 1.0, rtol=0, atol=1e-15)


# --------------------------------------------------------------- prolongation


@pytest.mark.parametrize("n", GRIDS_2D)
@pytest.mark.parametrize("bc", BCS_2D)
def test_face_prolongation_2d_is_the_printed_stencil(n, bc):
    o, lay, cl = _ctx(2, n, bc)
    P = _matrix(lambda v: o.prolong_add_faces(0, v), cl.nvel, lay.nvel)
    expect = np.zeros_like(P)
    for k, f, q in _faces(lay):
        if _is_wall(lay, k, f):
            continue
        t = 1 - k
        i, j = f[k], f[t]
        # coarse tangential rows: j even -> 3/4 on j/2, 1/4 on j/2 - 1 (printed);
        # j odd -> 3/4 on j/2, 1/4 on j/2 + 1 (mirror image)
        rows = [(j // 2, 3 / 4), (j // 2 - 1 if j % 2 == 0 else j // 2 + 1, 1 / 4)]
        # normal: i even -> the coarse face i/2; i odd -> 1/2 on i/2 and i/2 + 1
        # (printed: 3/8 = 1/2 * 3/4 and 1/8 = 1/2 * 1/4)
        cols = [(i // 2, 1.0)] if i % 2 == 0 else [(i // 2, 0.5), (i // 2 + 1, 0.5)]
        for (J, wt), (I, wn) in itertools.product(rows, cols):
            F = [0, 0, 0]
            F[k] = I
            sign = 1.0
            if lay.wall(t) and not (0 <= J < cl.n[t]):
                # missing neighbour behind a wall: reflect onto the face itself
                end = 0 if J < 0 else 1
                J = j // 2
                sign = -1.0 if W.end_is_noslip(lay.bc[t], end) else 1.0
            F[t] = J
            if _is_wall(cl, k, F):
                continue  # coarse wall faces are zero
            expect[q, _pos(cl, k, F)] += sign * wt * wn
    assert np.array_equal(P, expect)


def _linear_field(lay, h, coef, mask_fn=None):
    """u_k = coef[k][0] + coef[k][1:] . x at every stored face centre."""
    u = np.zeros(lay.nvel)
    for k, f, q in _faces(lay):
        x = _centre(k, f, h)
        u[q] = coef[k][0] + np.dot(coef[k][1:1 + 3], x)
    return u


LIN_GRIDS = [(2, (16, 16), (1, 1)), (2, (16, 8), (0, 0)), (2, (16, 16), (2, 3)),
             (3, (8, 8, 8), (1, 1, 1)), (3, (8, 8, 8), (0, 2, 1)), (3, (16, 8, 8), (0, 0, 0))]


def _inside(lay, k, f, margin_n, margin_t):
    """Faces whose transfer stencil stays away from walls and periodic
    seams: normal index in [margin_n, n - margin_n], tangential indices in
    [margin_t, n - 1 - margin_t]."""
    for a in range(lay.dim):
        if a == k:
            if not (margin_n <= f[a] <= lay.n[a] - margin_n):
                return False
        elif not (margin_t <= f[a] <= lay.n[a] - 1 - margin_t):
            return False
    return True


@pytest.mark.parametrize("dim,n,bc", LIN_GRIDS)
def test_face_transfers_reproduce_linear_fields(dim, n, bc):
    o, lay, cl = _ctx(dim, n, bc)
    h = 1.0 / lay.n[0]
    rng = np.random.default_rng(92)
    coef = rng.normal(size=(3, 4))
    if dim == 2:
        coef[:, 3] = 0.0
    uf = _linear_field(lay, h, coef)
    uc = _linear_field(cl, 2 * h, coef)
    Ru = o.restrict_faces(0, uf)
    Pu = o.prolong_add_faces(0, uc)
    nr = np_ = 0
    for k, F, qc in _faces(cl):
        if _is_wall(cl, k, F) or not _inside(cl, k, F, 1, 0):
            continue
        assert abs(Ru[qc] - uc[qc]) <= 1e-13, (k, F)
        nr += 1
    for k, f, q in _faces(lay):
        if _is_wall(lay, k, f) or not _inside(lay, k, f, 2, 1):
            continue
        assert abs(Pu[q] - uf[q]) <= 1e-13, (k, f)
        np_ += 1
    assert nr > 0 and np_ > 0


@pytest.mark.parametrize("dim,n", [(2, (16, 16)), (3, (8, 8, 8))])
def test_face_prolongation_wall_reflections(dim, n):
    """Along the tangent of a wall: a no-slip wall makes the fine row next to
    it take half its coarse value (odd reflection), so a field that vanishes
    linearly on the wall is reproduced; a free-slip wall reproduces a
    constant (even reflection).  Along the normal: the coarse wall face is
    zero, so a field vanishing linearly on the wall is reproduced at the
    first interior fine face."""
    h = 1.0 / n[0]
    for k in range(dim):
        for t in range(dim):
            if t == k:
                continue
            for kind, bcv in (("noslip", W.NOSLIP), ("freeslip", W.FREESLIP)):
                bc = [W.PERIODIC] * dim
                bc[t] = bcv
                o, lay, cl = _ctx(dim, n, tuple(bc))
                L = lay.n[t] * h
                for end in (0, 1):
                    def field(x):
                        if kind == "freeslip":
                            return 1.0
                        return x[t] if end == 0 else (L - x[t])
                    uc = np.zeros(cl.nvel)
                    for kk, F, qc in _faces(cl):
                        if kk == k:
                            uc[qc] = field(_centre(k, F, 2 * h))
                    Pu = o.prolong_add_faces(0, uc)
                    row = 0 if end == 0 else lay.n[t] - 1
                    checked = 0
                    for kk, f, q in _faces(lay):
                        if kk != k or f[t] != row or _is_wall(lay, k, f):
                            continue
                        if not _inside(lay, k, f, 2, -1):
                            continue
                        assert abs(Pu[q] - field(_centre(k, f, h))) <= 1e-13, (k, t, kind, end, f)
                        checked += 1
                    assert checked > 0
        # normal wall: u_k = x_k near the low wall, L - x_k near the high wall
        bc = [W.PERIODIC] * dim
        bc[k] = W.NOSLIP
        o, lay, cl = _ctx(dim, n, tuple(bc))
        L = lay.n[k] * h
        for end in (0, 1):
            uc = np.zeros(cl.nvel)
            for kk, F, qc in _faces(cl):
                if kk == k and not _is_wall(cl, k, F):
                    x = _centre(k, F, 2 * h)
                    uc[qc] = x[k] if end == 0 else L - x[k]
            Pu = o.prolong_add_faces(0, uc)
            i = 1 if end == 0 else lay.n[k] - 1
            for kk, f, q in _faces(lay):
                if kk == k and f[k] == i:
                    x = _centre(k, f, h)
                    assert abs(Pu[q] - (x[k] if end == 0 else L - x[k])) <= 1e-13


def test_face_prolongation_adds_to_its_target():
    o, lay, cl = _ctx(2, (8, 8), (1, 0))
    base = W.random_velocity(93, lay)
    base[lay.wall_mask()] = 0.0
    ec = W.random_velocity(94, cl)
    assert np.allclose(o.prolong_add_faces(0, ec, base),
                       base + o.prolong_add_faces(0, ec), rtol=0, atol=1e-15)


# --------------------------------------------------------------------- cells


@pytest.mark.parametrize("dim,n,bc", [(2, (8, 4), (0, 1)), (3, (4, 8, 4), (1, 0, 2))])
def test_cell_transfers_are_mean_and_injection(dim, n, bc):
    o, lay, cl = _ctx(dim, n, bc)
    R = _matrix(lambda v: o.restrict_cells(0, v), lay.ncell, cl.ncell)
    P = _matrix(lambda v: o.prolong_add_cells(0, v), cl.ncell, lay.ncell)
    fine = np.indices(lay.cell_shape).reshape(dim, -1)   # numpy axes: (z,) y, x
    cshape = cl.cell_shape
    parent = np.ravel_multi_index(tuple(fine[a] // 2 for a in range(dim)), cshape)
    expect_P = np.zeros_like(P)
    expect_P[np.arange(lay.ncell), parent] = 1.0
    assert np.array_equal(P, expect_P)
    assert np.array_equal(R, expect_P.T / 2 ** dim)
    # a linear field is restricted exactly (the children's centres average to
    # the parent's centre)
    h = 1.0 / lay.n[0]
    rng = np.random.default_rng(95)
    c = rng.normal(size=dim + 1)
    xf = [(fine[a] + 0.5) * h for a in range(dim)]
    cc = np.indices(cshape).reshape(dim, -1)
    xc = [(cc[a] + 0.5) * 2 * h for a in range(dim)]
    lin = lambda xs: c[0] + sum(c[1 + a] * xs[a] for a in range(dim))
    assert np.allclose(o.restrict_cells(0, lin(xf)), lin(xc), rtol=0, atol=1e-13)
