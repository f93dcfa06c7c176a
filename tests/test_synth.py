"""Pins for the synthetic layered-battery generator (inputs of every test).

The generator is checked against an independent face-loop assembly written
here in Python from the assembly rules, bit for bit, on tiny grids, and
against the structural counts the rules imply.
"""
import math

import numpy as np
import pytest

import synth


def _layer(t, N):
    for L, C in enumerate((1, 4, 6, 9, 10)):
        if (2 * t + 1) * 10 < 2 * N * C:
            return L
    return 4


def _harm(a, b):
    if a == 0.0 or b == 0.0:
        return 0.0
    return 2.0 * a * b / (a + b)


def face_loop_assembly(nx, ny, nz, nspecies, seed, j0=None):
    """Independent assembly: loops over cells and faces, dict accumulators."""
    dim = 3 if nz > 0 else 2
    nzz = nz if nz > 0 else 1
    nf = 3 + nspecies
    diff = (1e-3, 5e-4, 2e-3)
    ncell = nx * ny * nzz
    nl = ny if dim == 2 else nz
    u = synth.u01
    perm = [1e-3 * math.pow(1e-1 / 1e-3, u(seed, 0, c)) for c in range(ncell)]
    j0s = [0.1 * math.pow(10.0 / 0.1, u(seed, 1, c)) for c in range(ncell)] if j0 is None else list(j0)
    amp, kw, ph = [], [], []
    for m in range(4):
        amp.append(2.0 * u(seed, 3, 8 * m) - 1.0)
        kw.append([1 + int(3.0 * u(seed, 3, 8 * m + 1 + d)) for d in range(3)])
        ph.append(6.283185307179586 * u(seed, 3, 8 * m + 4))

    def coords(c):
        return (c % nx, (c // nx) % ny, c // (nx * ny))

    pt = []
    for c in range(ncell):
        x = coords(c)
        s = 0.0
        for m in range(4):
            arg = ph[m]
            for d in range(dim):
                arg += 6.283185307179586 * kw[m][d] * (x[d] + 0.5) / (nx, ny, nzz)[d]
            s += amp[m] * math.sin(arg)
        pt.append(s)

    def layer(c):
        x = coords(c)
        return _layer(x[1] if dim == 2 else x[2], nl)

    def kap(f, c):
        L = layer(c)
        if f == 0:
            return 1e4 if L in (0, 4) else (0.0 if L == 2 else 1e2)
        if f == 1:
            return 0.0 if L in (0, 4) else 1.0
        if f == 2:
            return perm[c]
        return diff[f - 3]

    def nb(c, q):
        x = list(coords(c))
        d, s = q // 2, (1 if q % 2 else -1)
        x[d] += s
        if x[d] < 0 or x[d] >= (nx, ny, nzz)[d]:
            return -1
        return x[0] + nx * (x[1] + ny * x[2])

    rows = []
    for c in range(ncell):
        L = layer(c)
        for f in range(nf):
            r = {}

            def add(col, v):
                r[col] = r[col] + v if col in r else v

            row = nf * c + f
            if (f == 0 and L == 2) or (f == 1 and L in (0, 4)):
                rows.append({row: 1.0})
                continue
            for q in range(2 * dim):
                n2 = nb(c, q)
                if n2 >= 0:
                    T = _harm(kap(f, c), kap(f, n2))
                    if T > 0.0:
                        add(row, T)
                        add(nf * n2 + f, -T)
                    if f >= 3:
                        uu = pt[c] - pt[n2]
                        add(row, max(uu, 0.0))
                        add(nf * n2 + f, -max(-uu, 0.0))
                else:
                    last = dim - 1
                    if (f == 0 and q == 2 * last) or (f == 2 and q == 2 * last + 1):
                        add(row, 2.0 * kap(f, c))
            if f >= 3:
                add(row, 100.0)
            if L in (1, 3):
                k = j0s[c]
                s_, e_ = nf * c, nf * c + 1
                if f == 0:
                    add(s_, k)
                    add(e_, -k)
                elif f == 1:
                    add(s_, -k)
                    add(e_, k)
                elif f >= 3:
                    add(s_, -0.5 * k)
                    add(e_, 0.5 * k)
            if f >= 3 and L not in (0, 4):
                for q in range(2 * dim):
                    n2 = nb(c, q)
                    if n2 < 0:
                        continue
                    Te = _harm(kap(1, c), kap(1, n2))
                    if Te > 0.0:
                        add(nf * c + 1, 0.1 * Te)
                        add(nf * n2 + 1, -(0.1 * Te))
            rows.append(r)
    rp = [0]
    ci, v = [], []
    for r in rows:
        for col in sorted(r):
            ci.append(col)
            v.append(r[col])
        rp.append(len(ci))
    return np.array(rp), np.array(ci), np.array(v)


@pytest.mark.parametrize("dims,nsp", [((4, 4, 0), 1), ((5, 3, 0), 1), ((4, 4, 3), 1), ((3, 3, 4), 3),
                                      ((4, 3, 10), 1)])
def test_face_loop_assembly_bit_exact(dims, nsp):
    nx, ny, nz = dims
    s = synth.make_system(nx, ny, nz, nsp, seed=77)
    rp, ci, v = face_loop_assembly(nx, ny, nz, nsp, 77)
    assert np.array_equal(s.rowptr, rp)
    assert np.array_equal(s.col, ci)
    assert np.array_equal(s.val.view(np.int64), v.view(np.int64))


def test_j0_override_and_derivative_map():
    s = synth.make_system(4, 3, 10, 1, seed=5)
    j0 = s.j0.copy()
    j0[s.layer == 1] *= 1.7
    s2 = synth.make_system(4, 3, 10, 1, seed=5, j0=j0)
    rp, ci, v = face_loop_assembly(4, 3, 10, 1, 5, j0=j0)
    assert np.array_equal(s2.val, v)
    # values are affine in j0 with slope dcoef on the entries of cell dcell
    dj = np.zeros(len(s.val))
    m = s.dcell >= 0
    dj[m] = (j0 - s.j0)[s.dcell[m]] * s.dcoef[m]
    assert np.allclose(s2.val - s.val, dj, rtol=1e-12, atol=1e-12)
    assert np.all(s.dcell[~m] == -1)


def _expected_nnz(nx, ny, nz, nsp):
    """Count of nonzeros implied by the rules, from face counts per field."""
    dim = 3 if nz > 0 else 2
    nzz = nz if nz > 0 else 1
    nl = ny if dim == 2 else nz
    layers = np.array([_layer(t, nl) for t in range(nl)])
    # per cell layer grid with the layered axis last
    shape = (nx, ny, nzz)
    idx = np.indices(shape)
    lay = layers[idx[1]] if dim == 2 else layers[idx[2]]
    active = {0: lay != 2, 1: (lay != 0) & (lay != 4)}
    total = 0
    nf = 3 + nsp

    def interior_faces(mask):
        cnt = 0
        for d in range(dim):
            a = np.take(mask, range(shape[d] - 1), axis=d)
            b = np.take(mask, range(1, shape[d]), axis=d)
            cnt += int(np.sum(a & b))
        return cnt

    allm = np.ones(shape, bool)
    ncell = nx * ny * nzz
    elec = int(np.sum((lay == 1) | (lay == 3)))
    for f in range(nf):
        if f in (0, 1):
            m = active[f]
            total += int(m.sum()) + 2 * interior_faces(m) + int((~m).sum())
        else:
            total += ncell + 2 * interior_faces(allm)
    total += 2 * elec  # phi_s <-> phi_e
    # species rows: phi_s column at electrode cells; phi_e columns (cell + active neighbours)
    m1 = active[1]
    for _ in range(nsp):
        total += elec
        total += int(m1.sum()) + 2 * interior_faces(m1)
    return total


@pytest.mark.parametrize("cfg,nnz", [(0, 24356), (1, 8610816)])
def test_config_sizes(cfg, nnz):
    c = synth.CONFIGS[cfg]
    assert _expected_nnz(c["nx"], c["ny"], c["nz"], c["nspecies"]) == nnz
    s = synth.make_system(cfg=cfg)
    assert s.nnz == nnz
    assert s.n == c["nx"] * c["ny"] * max(c["nz"], 1) * (3 + c["nspecies"])


@pytest.mark.parametrize("cfg", [2, 3, 4])
def test_config_sizes_formula(cfg):
    table = {2: 34588672, 3: 51758592, 4: 494798848}
    c = synth.CONFIGS[cfg]
    assert _expected_nnz(c["nx"], c["ny"], c["nz"], c["nspecies"]) == table[cfg]


def test_layers_and_rhs():
    # layer widths for the four layered-axis sizes used by the configurations
    exp = {32: (3, 10, 6, 10, 3), 64: (6, 20, 12, 20, 6), 96: (10, 28, 20, 28, 10), 128: (13, 38, 26, 38, 13)}
    for N, w in exp.items():
        got = np.bincount([synth._load().synth_layer(t, N) for t in range(N)], minlength=5)
        assert tuple(got) == w
    s = synth.make_system(6, 5, 8, 1, seed=3)
    # b = A x* recomputed in the same (ascending column) order is exact
    b2 = np.array([sum(s.val[k] * s.x_star[s.col[k]] for k in range(s.rowptr[i], s.rowptr[i + 1]))
                   for i in range(s.n)])
    assert np.array_equal(b2, s.b)


def test_block_symmetry_and_nonsingular():
    s = synth.make_system(5, 4, 6, 1, seed=11)
    import scipy.sparse as sp
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n)).toarray()
    f = s.field_of_row
    for fld in (0, 1, 2):
        B = A[np.ix_(f == fld, f == fld)]
        assert np.array_equal(B, B.T)
    # potentials pair block symmetric too (coupling +-k is symmetric)
    m = (f == 0) | (f == 1)
    V = A[np.ix_(m, m)]
    assert np.array_equal(V, V.T)
    # potentials do not depend on species or pressure: the upper-right block is zero
    assert not np.any(A[np.ix_(m, f >= 2)])
    sv = np.linalg.svd(A, compute_uv=False)
    assert sv[-1] > 1e-8 * sv[0]
