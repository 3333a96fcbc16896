"""GPU edge cases: every supported degree (p = 1 .. 6; p = 6 is the largest
whose FP64 workgroup fits in LDS) in both arithmetics, and the error paths
of the C ABI that guard a launch (every bad argument is rejected on the
host before any kernel runs)."""
import ctypes as C

import numpy as np
import pytest

from paper_2502_17805_amd import inputs as inp

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def sd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_17805_amd import sdmhd
    return sdmhd


@pytest.mark.parametrize("p", [1, 2, 4, 6])
def test_every_degree_residual_and_step(sd, oracle, p):
    import torch
    print(f"degree p={p}", flush=True)
    ml = sd.shell(2, 1, p)
    mo = oracle.Mesh.shell(p + 1, 2, 1)
    bg = inp.Background(3.0)
    Q = inp.shell_state(ml.x_sp, bg, 5)
    pr = inp.run_params(5, bg)
    ch = inp.glm_speed(Q)
    pr.update(c_h=ch, glm_a=ch / (bg.rt - bg.rb))
    pg, po = sd.make_params(**pr), oracle.make_params(**pr)
    s = sd.Solver(ml)
    Rg = s.residual(pg, torch.from_numpy(Q).cuda()).cpu().numpy()
    Ro, ts = mo.residual(po, Q, with_scale=True)
    assert (np.abs(Rg - Ro).max(axis=(0, 2)) <= TOL * ts).all()
    dt = inp.time_step(Q, ml.Sj_sp, ch, 0.1)
    s.set_state(Q)
    s.step(pg, dt)
    qo = mo.step(po, Q, dt)
    err = np.abs(s.state.cpu().numpy() - qo).max(axis=(0, 2))
    assert (err <= TOL * (np.abs(qo).max(axis=(0, 2)) + dt * ts)).all()
    # FP32-mixed at this degree: the residual within the mixed bound (1e-5 of
    # the term scale) and the step's FP64 accumulation around it
    m32 = sd.Solver(ml, arith=1)
    R32 = m32.residual(pg, torch.from_numpy(Q).cuda()).cpu().numpy()
    assert (np.abs(R32 - Ro).max(axis=(0, 2)) <= 1e-5 * ts).all()
    m32.set_state(Q)
    m32.step(pg, dt)
    err = np.abs(m32.state.cpu().numpy() - qo).max(axis=(0, 2))
    assert (err <= 1e-5 * (np.abs(qo).max(axis=(0, 2)) + dt * ts)).all()


def _ctx(sd, p=3, arith=0):
    h = C.c_void_p()
    assert sd._lib.sdm_create(0, p, arith, C.byref(h)) == sd.SDM_OK
    return h


def test_create_rejects_unsupported_degree(sd):
    h = C.c_void_p()
    for p, arith in ((0, 0), (7, 0), (3, 2)):
        assert sd._lib.sdm_create(0, p, arith, C.byref(h)) != sd.SDM_OK
        assert sd._lib.sdm_last_error()


def test_mesh_bind_rejects_empty_and_corrupt_tables(sd):
    import torch
    m = sd.shell(1, 1, 3)
    dev = {k: torch.from_numpy(np.ascontiguousarray(getattr(m, k))).cuda()
           for k in ("x_sp", "detJ", "S_fp", "Sj_sp", "nbr", "n_face")}
    h = _ctx(sd)
    try:
        def desc(E, NB, nbr):
            return sd.MeshDesc(E, NB, dev["x_sp"].data_ptr(), dev["detJ"].data_ptr(), dev["S_fp"].data_ptr(),
                               dev["Sj_sp"].data_ptr(), nbr.data_ptr(), dev["n_face"].data_ptr())
        assert sd._lib.sdm_mesh_bind(h, C.byref(desc(0, 0, dev["nbr"]))) != sd.SDM_OK
        # past the largest mesh the element index fields can address (checked
        # before the table is read)
        assert sd._lib.sdm_mesh_bind(h, C.byref(desc(1 << 25, m.NB, dev["nbr"]))) != sd.SDM_OK
        for bad in (m.E << 6, -(1 + 3 + 4 * m.NB), -(1 + 4 * m.NB)):  # element, import face, wall face
            nb = dev["nbr"].clone()
            nb[0, 0] = int(bad)
            assert sd._lib.sdm_mesh_bind(h, C.byref(desc(m.E, m.NB, nb))) != sd.SDM_OK, bad
        assert sd._lib.sdm_mesh_bind(h, C.byref(desc(m.E, m.NB, dev["nbr"]))) == sd.SDM_OK
        nb = C.c_size_t()
        assert sd._lib.sdm_workspace_size(h, C.byref(nb)) == sd.SDM_OK and nb.value > 0
    finally:
        sd._lib.sdm_destroy(h)


def test_dirichlet_mesh_requires_ghost(sd):
    import torch
    m = sd.box(3, 3, 2, 3, periodic=3)  # the z faces are boundary faces
    s = sd.Solver(m)
    Q = torch.from_numpy(inp.smooth_random_state(m.x_sp, 1)).cuda()
    s.residual(sd.make_params(c_h=1.0), Q)  # as walls: no ghost state needed
    with pytest.raises(sd.SdmError):  # as Dirichlet faces: the ghost state is required
        s.residual(sd.make_params(c_h=1.0, wall_kind=(1, 1)), Q)


def test_batch_rejects_empty_and_mismatched(sd):
    nb = C.c_size_t()
    assert sd._lib.sdm_batch_workspace_size(0, C.byref(nb)) != sd.SDM_OK
    items = (sd.BatchItem * 1)()
    assert sd._lib.sdm_batch_stage(items, 0, None, 0, 0, None) != sd.SDM_OK


def test_mixed_geometry_copy_follows_rebind(sd):
    """FP32-mixed reads the FP32 geometry copies sdm_mesh_bind makes: a
    rebind of the same arrays gives bitwise the same residual; arrays
    changed in place are not seen until the next bind, after which the
    residual equals a fresh context's on the new geometry."""
    import torch
    print("mixed geometry rebind", flush=True)
    ma, mb = sd.shell(2, 1, 3, 0.70, 0.98), sd.shell(2, 1, 3, 0.60, 0.95)
    bg = inp.Background(3.0)
    Q = torch.from_numpy(inp.shell_state(ma.x_sp, bg, 4)).cuda()
    prm = sd.make_params(**inp.run_params(4, bg), c_h=1.0)
    s = sd.Solver(ma, arith=1)

    def rebind():
        md = sd.MeshDesc(ma.E, ma.NB, s.x_sp.data_ptr(), s.detJ.data_ptr(), s.S_fp.data_ptr(),
                         s.Sj_sp.data_ptr(), s.nbr.data_ptr(), s.n_face.data_ptr())
        sd._check(sd._lib.sdm_mesh_bind(s._h, C.byref(md)))

    r1 = s.residual(prm, Q).clone()
    rebind()
    assert torch.equal(s.residual(prm, Q), r1)
    for k in ("x_sp", "detJ", "S_fp", "Sj_sp", "n_face"):
        getattr(s, k).copy_(torch.from_numpy(np.ascontiguousarray(getattr(mb, k))))
    assert torch.equal(s.residual(prm, Q), r1)  # the copies made at the last bind
    rebind()
    r2 = s.residual(prm, Q)
    ref = sd.Solver(mb, arith=1).residual(prm, Q)
    assert not torch.equal(r2, r1)
    assert torch.equal(r2, ref)
