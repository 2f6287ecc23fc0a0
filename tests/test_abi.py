"""The C-ABI library loads on the host and exports every symbol that
include/ctmhd.h declares; argument validation happens before any device call."""
import ctypes
import os
import re

import pytest

from paper_2609_10816_amd import ctmhd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ctmhd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ctmhd_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported():
    names = _declared()
    assert "ctmhd_step" in names and "ctmhd_step_batched" in names and "ctmhd_step_adjoint" in names
    L = ctypes.CDLL(ctmhd.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(ctmhd.EXPORTED) == set(names)


def test_required_ghosts():
    for recon, g in [("pc", 2), ("plm", 3), ("plm_minmod", 3), ("ppm", 4)]:
        assert ctmhd.required_ghosts(ctmhd.make_params(recon=recon)) == g


def test_box_elems_and_workspace():
    p = ctmhd.make_params(recon="ppm")
    b = ctmhd.make_box((10, 7, 3), 4, (0.1, 0.2, 0.3))
    assert ctmhd.lib().ctmhd_box_elems(ctypes.byref(b)) == 18 * 15 * 11
    ws64 = ctmhd.workspace_bytes(p, b)
    ws32 = ctmhd.workspace_bytes(ctmhd.make_params(recon="ppm", precision="fp32"), b)
    assert ws64 > ws32 > 0


def test_workspace_holds_the_stored_first_steps():
    # B25a (12 arrays) and FS18 (18 arrays) store the first step of their
    # two-step corner reconstructions with PPM only; one array per element of
    # the ghosted box in the stencil type, 256-byte aligned
    b = ctmhd.make_box((10, 7, 3), 4, (0.1, 0.2, 0.3))
    e = 18 * 15 * 11
    for prec, tb in (("fp64", 8), ("fp32", 4)):
        one = -(-e * tb // 256) * 256
        ws = {(r, emf): ctmhd.workspace_bytes(ctmhd.make_params(recon=r, emf=emf, precision=prec), b)
              for r in ("plm", "ppm") for emf in ("q26", "b25a", "fs18")}
        assert ws[("plm", "b25a")] == ws[("plm", "fs18")] == ws[("plm", "q26")] + 3 * one
        assert ws[("ppm", "b25a")] == ws[("ppm", "q26")] + (3 + 12) * one
        assert ws[("ppm", "fs18")] == ws[("ppm", "q26")] + (3 + 18) * one


def _call_step(p, b, nsteps=1):
    L = ctmhd.lib()
    dummy = ctypes.c_void_p(256)  # never dereferenced: validation fails first
    cons = ctmhd._PTR5(*([dummy.value] * 5))
    bf = ctmhd._PTR3(*([dummy.value] * 3))
    return L.ctmhd_step(ctypes.byref(p), ctypes.byref(b), cons, bf, nsteps, None, None, None,
                        None, 0, None)


@pytest.mark.parametrize("bad", [
    dict(gamma=1.0), dict(eta=-1.0), dict(cfl=0.0), dict(cfl=1.2), dict(eta=1e-3, cfl=0.4),
])
def test_bad_params_rejected(bad):
    kw = dict(recon="plm")
    kw.update(bad)
    p = ctmhd.make_params(**kw)
    b = ctmhd.make_box((8, 8, 8), 3, (0.1, 0.1, 0.1))
    assert _call_step(p, b) == -1
    assert ctmhd.lib().ctmhd_last_error()


def test_bad_box_rejected():
    p = ctmhd.make_params(recon="ppm")
    assert _call_step(p, ctmhd.make_box((8, 8, 8), 3, (0.1, 0.1, 0.1))) == -1  # ng < 4
    assert b"ghost" in ctmhd.lib().ctmhd_last_error()
    assert _call_step(p, ctmhd.make_box((8, 0, 8), 4, (0.1, 0.1, 0.1))) == -1
    assert _call_step(p, ctmhd.make_box((8, 8, 8), 4, (0.1, -1.0, 0.1))) == -1
    # workspace missing
    assert _call_step(p, ctmhd.make_box((8, 8, 8), 4, (0.1, 0.1, 0.1))) == -1
    assert b"workspace" in ctmhd.lib().ctmhd_last_error()


def test_precision_forms():
    b = ctmhd.make_box((8, 8, 8), 3, (0.1,) * 3)
    for prec in ("fp64", "fp32", "fp32_r64"):
        assert _call_step(ctmhd.make_params(precision=prec), b) == -1
        assert b"workspace" in ctmhd.lib().ctmhd_last_error()
    # both FP32 forms keep their stencil arrays in float32
    bw = ctmhd.make_box((10, 7, 3), 4, (0.1, 0.2, 0.3))
    assert (ctmhd.workspace_bytes(ctmhd.make_params(recon="ppm", precision="fp32"), bw) ==
            ctmhd.workspace_bytes(ctmhd.make_params(recon="ppm", precision="fp32_r64"), bw))
    p = ctmhd.make_params()
    for bad in (3, -1):
        p.precision = bad
        assert _call_step(p, b) == -1
        assert b"precision" in ctmhd.lib().ctmhd_last_error()


def test_unsupported_averaging():
    p = ctmhd.make_params()
    p.emf_average = 1
    assert _call_step(p, ctmhd.make_box((8, 8, 8), 3, (0.1,) * 3)) == -2


def test_tile_knob_validation():
    b = ctmhd.make_box((8, 8, 8), 3, (0.1,) * 3)
    ok = ctmhd.make_params(tile=ctmhd.make_tile(chunk=16, strips=2, xrows=8))
    assert _call_step(ok, b) == -1  # passes the knob check, stops at the missing workspace
    assert b"workspace" in ctmhd.lib().ctmhd_last_error()
    for m in ("contiguous", "banded"):
        p = ctmhd.make_params(tile=ctmhd.make_tile(xcd_map=m))
        assert _call_step(p, b) == -1 and b"workspace" in ctmhd.lib().ctmhd_last_error()
    for k in ("edge", "march"):
        p = ctmhd.make_params(tile=ctmhd.make_tile(emf_kernel=k, persistent=True))
        assert _call_step(p, b) == -1 and b"workspace" in ctmhd.lib().ctmhd_last_error()
    for bad in (1 << 17, 1 << 18, 3 << 19, 3 << 21, 1 << 23, -1):
        p = ctmhd.make_params(tile=bad)
        assert _call_step(p, b) == -1
        assert b"tile" in ctmhd.lib().ctmhd_last_error()


def test_adjoint_configurations_and_workspace_query():
    b = ctmhd.make_box((8, 8, 8), 4, (0.1,) * 3)
    for kw in (dict(recon="pc"), dict(recon="plm"), dict(recon="plm_minmod"), dict(recon="ppm"),
               dict(recon="ppm", riemann="llf"), dict(recon="plm", eta=1e-3, cfl=0.3),
               dict(recon="ppm", emf="b25a"), dict(recon="pc", riemann="llf", emf="b25a"),
               dict(recon="plm", emf="fs18")):
        p = ctmhd.make_params(fofc=False, **kw)
        assert ctmhd.adjoint_workspace_bytes(p, b) > ctmhd.workspace_bytes(p, b), kw
    for kw in (dict(precision="fp32"), dict(precision="fp32_r64")):
        assert ctmhd.adjoint_workspace_bytes(ctmhd.make_params(**kw), b) == 0, kw
        assert b"adjoint" in ctmhd.lib().ctmhd_last_error()


def test_adjoint_rejects_null_pointers_before_any_device_call():
    L = ctmhd.lib()
    p = ctmhd.make_params(recon="plm", fofc=False)
    b = ctmhd.make_box((8, 8, 8), 3, (0.1,) * 3)
    d = 256  # never dereferenced: validation fails first
    c5 = ctmhd._PTR5(*([d] * 5))
    c3 = ctmhd._PTR3(*([d] * 3))
    rc = L.ctmhd_step_adjoint(ctypes.byref(p), ctypes.byref(b), c5, c3, None, c5, c3, c5, c3,
                              None, 0, None)
    assert rc == -1
    assert b"NULL" in L.ctmhd_last_error()
