"""CPU checks of the C ABI: the library loads, exports every function that
include/cr_solver.h declares, and rejects invalid arguments on the host before
any device work (CR_EINVAL / CR_ENOMEM paths)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "cr_solver.h")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(cr_[a-z_0-9]+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def cr():
    from paper_2607_11340_amd import crsolver
    return crsolver


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("cr_fk", "cr_cost_grad", "cr_solve_ik", "cr_select_top", "cr_status_string", "cr_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol(cr):
    out = subprocess.run(["nm", "-D", "--defined-only", cr.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (cr_[a-z_0-9]+)$", out, flags=re.M))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    for f in declared_functions():
        assert hasattr(cr.lib, f)


def test_status_strings(cr):
    for s in range(5):
        assert cr.lib.cr_status_string(s).startswith(b"CR_")


def _robot(cr, **kw):
    base = dict(L=[0.1, 0.08, 0.06], r=[0.01, 0.008, 0.006], u_max=[0.008] * 3)
    base.update(kw)
    return cr.Robot(**base)


def test_fk_rejects_bad_arguments_on_host(cr):
    L = cr.lib
    for bad in (dict(L=[0.1, -0.08, 0.06]), dict(r=[0.01, 0.0, 0.006]), dict(L=[0.1] * 7, r=[0.01] * 7, u_max=[1.0] * 7)):
        rb = _robot(cr, **bad).c() if len(bad.get("L", [0] * 3)) <= 6 else None
        if rb is None:
            rb = cr._Robot()
            rb.n_seg = 7
        rc = L.cr_fk(C.byref(rb), 10, C.c_void_p(1), 10, None, None, None, 0, None)
        assert rc == cr.CR_EINVAL
        assert L.cr_last_error()
    rb = _robot(cr).c()
    assert L.cr_fk(None, 10, C.c_void_p(1), 10, None, None, None, 0, None) == cr.CR_EINVAL
    assert L.cr_fk(C.byref(rb), 10, C.c_void_p(1), 5, None, None, None, 0, None) == cr.CR_EINVAL  # ld < B
    assert L.cr_fk(C.byref(rb), 10, None, 10, None, None, None, 0, None) == cr.CR_EINVAL  # u NULL
    assert L.cr_fk(C.byref(rb), 10, C.c_void_p(1), 10, None, None, None, 7, None) == cr.CR_EINVAL  # dtype


def test_solve_ik_rejects_bad_arguments_on_host(cr):
    L = cr.lib
    rb, wc, sc = _robot(cr).c(), cr.Weights().c(), cr._Spheres(0, 0, None, 0)
    p = C.c_void_p(1)

    def call(P=4, S=8, opts=None, weights=None, ws=None, ws_bytes=0, dtype=0, arrays=True):
        oc = (opts or cr.Opts()).c()
        w = (weights or cr.Weights()).c()
        a = p if arrays else None
        return L.cr_solve_ik(C.byref(rb), C.byref(sc), P, a, S, a, C.byref(w), C.byref(oc), a, a, a, ws, ws_bytes,
                             dtype, None)

    assert call(S=0) == cr.CR_EINVAL
    assert call(S=5000) == cr.CR_EINVAL
    assert call(P=-1) == cr.CR_EINVAL
    assert call(opts=cr.Opts(n_final=65)) == cr.CR_EINVAL
    assert call(opts=cr.Opts(ls_max=0)) == cr.CR_EINVAL
    assert call(opts=cr.Opts(lambda0=0.0)) == cr.CR_EINVAL
    assert call(weights=cr.Weights(dt=0.0)) == cr.CR_EINVAL
    assert call(weights=cr.Weights(rho_lim=float("nan"))) == cr.CR_EINVAL
    assert call(arrays=False) == cr.CR_EINVAL
    assert call(P=0) == cr.CR_OK  # empty batch: nothing to do
    oc = cr.Opts().c()
    need = L.cr_solve_ik_workspace(C.byref(rb), 4, 8, C.byref(oc), 0)
    assert need > 0
    assert call(ws=C.c_void_p(4096), ws_bytes=need - 1) == cr.CR_ENOMEM
    assert call(ws=C.c_void_p(4096 + 16), ws_bytes=need) == cr.CR_EINVAL  # not 256-byte aligned
    assert "aligned" in L.cr_last_error().decode()


def test_workspace_size_scales(cr):
    L = cr.lib
    rb, oc = _robot(cr).c(), cr.Opts().c()
    a = L.cr_solve_ik_workspace(C.byref(rb), 100, 64, C.byref(oc), 0)
    b = L.cr_solve_ik_workspace(C.byref(rb), 200, 64, C.byref(oc), 0)
    c = L.cr_solve_ik_workspace(C.byref(rb), 100, 64, C.byref(oc), 1)
    assert 0 < a < b and a < c
    assert L.cr_solve_ik_workspace(C.byref(rb), 100, 0, C.byref(oc), 0) == 0


def test_select_top_rejects_bad_arguments_on_host(cr):
    L = cr.lib
    p = C.c_void_p(1)
    assert L.cr_select_top(4, 0, 2, p, p, p, None, 2, 1e-3, p, 0, None) == cr.CR_EINVAL
    assert L.cr_select_top(4, 8, 2, p, p, p, None, 0, 1e-3, p, 0, None) == cr.CR_EINVAL
    assert L.cr_select_top(4, 8, 2, p, p, p, None, 65, 1e-3, p, 0, None) == cr.CR_EINVAL
    assert L.cr_select_top(4, 8, 2, p, p, p, None, 2, -1.0, p, 0, None) == cr.CR_EINVAL
    assert L.cr_select_top(4, 8, 2, p, None, p, None, 2, 1e-3, p, 0, None) == cr.CR_EINVAL


def test_batch_table_validation_on_host(cr):
    """cr_solve_batch rejects malformed tables before any device work; the
    workspace query is host-only and grows with the table."""
    L = cr.lib
    rob = (cr._Robot * 2)(_robot(cr).c(), _robot(cr, L=[0.1], r=[0.01], u_max=[0.01]).c())
    wc = (cr._Weights * 3)(*[cr.Weights().c()] * 3)
    oc = (cr._Opts * 3)(*[cr.Opts().c()] * 3)
    p = C.c_void_p(1)

    def table(rows):
        t = (cr._Problem * len(rows))()
        for i, (kind, robot, H, S, M) in enumerate(rows):
            t[i].kind, t[i].robot, t[i].H, t[i].S, t[i].n_sph = kind, robot, H, S, M
        return t

    good = [(0, 0, 0, 16, 0), (1, 1, 5, 8, 2), (2, 0, 3, 4, 0)]
    for bad in ([(3, 0, 0, 16, 0)], [(0, 2, 0, 16, 0)], [(0, 0, 1, 16, 0)], [(2, 0, 0, 4, 0)], [(1, 0, 256, 4, 0)],
                [(0, 0, 0, 0, 0)], [(0, 0, 0, 4097, 0)], [(0, 0, 0, 16, 513)], [(0, 0, 0, 16, -1)]):
        t = table(good + bad)
        rc = L.cr_solve_batch(rob, 2, t, len(good) + 1, p, p, p, wc, oc, p, p, p, None, 0, 0, 0, None)
        assert rc == cr.CR_EINVAL, bad
        assert L.cr_solve_batch_workspace(rob, 2, t, len(good) + 1, oc, 0) == 0
    t = table(good)
    t[0].task_off = -1
    assert L.cr_solve_batch(rob, 2, t, 3, p, p, p, wc, oc, p, p, p, None, 0, 0, 0, None) == cr.CR_EINVAL
    assert L.cr_solve_batch(rob, 0, table(good), 3, p, p, p, wc, oc, p, p, p, None, 0, 0, 0, None) == cr.CR_EINVAL
    # graph mode needs a caller workspace
    assert L.cr_solve_batch(rob, 2, table(good), 3, p, p, p, wc, oc, p, p, p, None, 0, 0, 1, None) == cr.CR_EINVAL
    # too small a workspace
    w4k = C.c_void_p(4096)
    assert L.cr_solve_batch(rob, 2, table(good), 3, p, p, p, wc, oc, p, p, p, w4k, 16, 0, 0, None) == cr.CR_ENOMEM
    # a misaligned workspace
    assert L.cr_solve_batch(rob, 2, table(good), 3, p, p, p, wc, oc, p, p, p, p, 1 << 30, 0, 0, None) == cr.CR_EINVAL
    a = L.cr_solve_batch_workspace(rob, 2, table(good), 3, oc, 0)
    b = L.cr_solve_batch_workspace(rob, 2, table(good + good), 6, oc, 0)
    c = L.cr_solve_batch_workspace(rob, 2, table(good), 3, oc, 1)
    assert 0 < a < b and a < c


def test_prm_rejects_bad_arguments_on_host(cr):
    L = cr.lib
    rb = _robot(cr).c()
    sp = cr._Spheres()
    fake = C.c_void_p(256)
    for bad in (dict(n_nodes=0), dict(n_nodes=4096), dict(k=0), dict(k=33), dict(n_check=65), dict(max_attempts=0)):
        o = cr.PrmOpts(**{**dict(n_nodes=64, k=4, n_check=2), **bad}).c()
        assert L.cr_prm_build(C.byref(rb), C.byref(sp), 4, C.byref(o), fake, fake, fake, fake, fake, fake,
                              None) == cr.CR_EINVAL
    o = cr.PrmOpts(n_nodes=64, k=4, n_check=2).c()
    assert L.cr_prm_build(C.byref(rb), C.byref(sp), 70000, C.byref(o), fake, fake, fake, fake, fake, fake,
                          None) == cr.CR_EINVAL
    assert L.cr_prm_build(C.byref(rb), C.byref(sp), 4, C.byref(o), None, fake, fake, fake, fake, fake,
                          None) == cr.CR_EINVAL
    ext = _robot(cr, L_min=[0.05, 0.04, 0.03], L_max=[0.12, 0.1, 0.08]).c()
    assert L.cr_prm_build(C.byref(ext), C.byref(sp), 4, C.byref(o), fake, fake, fake, fake, fake, fake,
                          None) == cr.CR_EUNSUPPORTED
    for H, S in ((0, 4), (256, 4), (8, 0), (8, 4097)):
        assert L.cr_prm_query(C.byref(rb), C.byref(sp), 4, C.byref(o), fake, fake, fake, fake, fake, fake, H, S, None,
                              0, fake, fake, None, None) == cr.CR_EINVAL
    # the roadmap may be missing only for the straight-line initializer
    assert L.cr_prm_query(C.byref(rb), C.byref(sp), 4, C.byref(o), None, None, None, None, None, fake, 8, 4, None, 0,
                          fake, fake, None, None) == cr.CR_EINVAL
    assert L.cr_prm_query(C.byref(rb), C.byref(sp), 4, C.byref(o), None, None, None, None, None, fake, 8, 4, None, 2,
                          fake, fake, None, None) == cr.CR_EINVAL


def header_constants():
    src = re.sub(r"/\*.*?\*/", "", open(HDR).read(), flags=re.S)
    return {k: int(v) for k, v in re.findall(r"\b(CR_[A-Z_0-9]+)\s*=\s*(\d+)", src)}


def test_binding_constants_match_the_header(cr):
    """The binding's enum values and flag bits are the header's."""
    h = header_constants()
    assert (cr.F32, cr.F64) == (h["CR_F32"], h["CR_F64"])
    assert cr.KIND == {"ik": h["CR_KIND_IK"], "path": h["CR_KIND_PATH"], "traj": h["CR_KIND_TRAJ"]}
    assert (cr.SOLVED, cr.LIMIT_VIOLATION, cr.COLLISION, cr.NONFINITE, cr.NOT_CONVERGED) == (
        h["CR_SOLVED"], h["CR_LIMIT_VIOLATION"], h["CR_COLLISION"], h["CR_NONFINITE"], h["CR_NOT_CONVERGED"])
    assert (cr.BATCH_GRAPH, cr.BATCH_PERSISTENT) == (h["CR_BATCH_GRAPH"], h["CR_BATCH_PERSISTENT"])
    assert cr.BATCH_GRAPH & cr.BATCH_PERSISTENT == 0
