"""Pins of the oracle's mesh, metrics and face table (paper, Sec. "Meshing" and
Sec. "Spectral Difference Method": mapping P, Jacobi matrix, Eq. G.E. comp)."""
import numpy as np
import pytest


def _fam_line(N, d, fp_vals):
    """reshape family-d flux-point values [(N+1)N^2] to [line(a,b)][f]"""
    if d == 0:
        v = fp_vals.reshape(N, N, N + 1)           # [b][a][f]
        return v.reshape(N * N, N + 1)
    if d == 1:
        v = fp_vals.reshape(N, N + 1, N)           # [b][f][a]
        return v.transpose(0, 2, 1).reshape(N * N, N + 1)
    v = fp_vals.reshape(N + 1, N, N)               # [f][b][a]
    return v.transpose(1, 2, 0).reshape(N * N, N + 1)


def _sp_lines(N, d, sp_vals):
    v = sp_vals.reshape(N, N, N)                   # [c][b][a]
    if d == 0:
        return v.reshape(N * N, N)
    if d == 1:
        return v.transpose(0, 2, 1).reshape(N * N, N)
    return v.transpose(1, 2, 0).reshape(N * N, N)


@pytest.mark.parametrize("Nz,Nr", [(1, 1), (2, 2), (3, 2)])
def test_counts(oracle, Nz, Nr):
    m = oracle.Mesh.shell(6, Nz, Nr)
    E = 6 * Nr * Nz * Nz
    assert m.E == E                                 # N_cells = 6 N_r N_z^2 (Sec. Meshing)
    assert m.F == (6 * E + 12 * Nz * Nz) // 2
    assert m.NB == 12 * Nz * Nz


def test_jacobian_positive_and_volume_converges(oracle):
    exact = 4.0 / 3.0 * np.pi * (0.98 ** 3 - 0.70 ** 3)
    errs = []
    for Nz in (1, 2, 4):
        m = oracle.Mesh.shell(6, Nz, 1)
        assert m.get("detJ_sp").min() > 0
        errs.append(abs(m.get("W3detJ").sum() - exact) / exact)
    assert errs[-1] < 1e-8 and errs[0] > errs[1] > errs[2]


@pytest.mark.parametrize("N", [4, 6])
def test_discrete_gcl(oracle, N):
    """sum_d D_d S^d = 0 at every solution point (what free-stream needs)."""
    m = oracle.Mesh.shell(N, 2, 1)
    _, _, _, D, _ = oracle.tables(N)
    S = m.get("S_fp")
    E = m.E
    div = np.zeros((E, 3, N ** 3))
    for e in range(E):
        for x in range(3):
            acc = np.zeros(N ** 3)
            for d in range(3):
                lines = _fam_line(N, d, S[e, d, x])                 # [line][f]
                dl = lines @ D.T                                    # [line][i]
                # scatter back to SP layout
                sp = np.zeros((N * N, N))
                sp[:] = dl
                if d == 0:
                    acc += sp.reshape(N ** 3)
                elif d == 1:
                    acc += sp.reshape(N, N, N).transpose(0, 2, 1).reshape(N ** 3)
                else:
                    acc += sp.reshape(N, N, N).transpose(2, 0, 1).reshape(N ** 3)
            div[e, x] = acc
    scale = np.abs(S).max()
    assert np.abs(div).max() < 1e-12 * scale
    # the pin is not vacuous: a perturbed metric breaks it
    assert np.abs(_fam_line(N, 0, S[0, 0, 0] * 1.001) @ D.T - _fam_line(N, 0, S[0, 0, 0]) @ D.T).max() > 1e-8 * scale


def test_metric_matches_jacobian(oracle):
    """S^d at SPs equals |J| times row d of J^-1 (cofactors of the map's
    Jacobian) up to truncation; exact for an affine box."""
    m = oracle.Mesh.box(4, 3, 3, 3, L=(1.0, 2.0, 0.5), periodic=0)
    S = m.get("S_sp")
    dj = m.get("detJ_sp")
    h = np.array([1.0 / 3, 2.0 / 3, 0.5 / 3])
    np.testing.assert_allclose(dj, h.prod(), rtol=1e-13)
    for d in range(3):
        for x in range(3):
            want = (h.prod() / h[d]) if d == x else 0.0
            np.testing.assert_allclose(S[:, d, x], want, atol=1e-13)


@pytest.mark.parametrize("N,Nz,Nr", [(6, 2, 2), (4, 3, 1)])
def test_faces_watertight_normals(oracle, N, Nz, Nr):
    """At every interior face point the two sides' outward metric normals are
    opposite (orientation codes pair up the same physical points)."""
    m = oracle.Mesh.shell(N, Nz, Nr)
    S = m.get("S_fp")
    faces = m.get("faces")

    def fp_index(d, f, a, b):
        if d == 0:
            return f + (N + 1) * (a + N * b)
        if d == 1:
            return a + N * (f + (N + 1) * b)
        return a + N * (b + N * f)

    def omap(o, a, b):
        p, q = (b, a) if o & 4 else (a, b)
        return (N - 1 - p if o & 1 else p), (N - 1 - q if o & 2 else q)

    worst = 0.0
    n_orient = set()
    for eL, fL, eR, fR, o in faces:
        if eR < 0:
            continue
        n_orient.add(int(o))
        for b in range(N):
            for a in range(N):
                a2, b2 = omap(o, a, b)
                sL = (1 if fL % 2 else -1) * S[eL, fL // 2, :, fp_index(fL // 2, N if fL % 2 else 0, a, b)]
                sR = (1 if fR % 2 else -1) * S[eR, fR // 2, :, fp_index(fR // 2, N if fR % 2 else 0, a2, b2)]
                worst = max(worst, np.abs(sL + sR).max() / np.abs(sL).max())
    assert worst < 1e-12
    assert len(n_orient) > 1  # the shell really exercises non-trivial orientations


def test_boundary_points_on_spheres(oracle):
    m = oracle.Mesh.shell(6, 2, 2)
    xb = m.get("x_bfp")
    r = np.sqrt((xb ** 2).sum(axis=1))
    faces = m.get("faces")
    bf = faces[faces[:, 2] < 0]
    for eL, fL, g, bi, _ in bf:
        want = 0.70 if g == -1 else 0.98
        # the isoparametric map interpolates the sphere: r exact at the nodes, close between
        assert np.abs(r[bi] - want).max() < 2e-6
