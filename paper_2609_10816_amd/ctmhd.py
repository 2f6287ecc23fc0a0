"""Python binding of libctmhd (ctypes).  Argument marshalling only: every step
of the method runs in the HIP kernels of the library.  PyTorch provides the
device memory and the stream.

The library must have been built (``python -m paper_2609_10816_amd.build`` or
``__graft_entry__.build()``); without it every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctmhd.so")

RECON = {"pc": 0, "plm": 1, "plm_mc": 1, "plm_minmod": 2, "ppm": 3}
RIEMANN = {"hlld": 0, "llf": 1}
EMF = {"q26": 0, "b25a": 1, "fs18": 2}
PRECISION = {"fp64": 0, "fp32": 1, "fp32_r64": 2}
DT_GLOBAL, DT_PER_BOX = 0, 1


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("eta", ctypes.c_double), ("cfl", ctypes.c_double),
                ("recon", ctypes.c_int32), ("riemann", ctypes.c_int32),
                ("emf_compute", ctypes.c_int32), ("emf_average", ctypes.c_int32),
                ("fofc", ctypes.c_int32), ("flag_criteria", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("force_flags", ctypes.c_void_p)]


class Box(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ng", ctypes.c_int32), ("dx", ctypes.c_double * 3),
                ("offset", ctypes.c_int64)]


_lib = None
_P = ctypes.POINTER(Params)
_B = ctypes.POINTER(Box)
_vp = ctypes.c_void_p
_PTR5 = ctypes.c_void_p * 5
_PTR3 = ctypes.c_void_p * 3


class CtmhdError(RuntimeError):
    pass


def lib():
    """Load libctmhd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CtmhdError(f"{LIB_PATH} is missing: build it first (paper_2609_10816_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        L.ctmhd_required_ghosts.argtypes = [_P]
        L.ctmhd_required_ghosts.restype = ctypes.c_int
        L.ctmhd_box_elems.argtypes = [_B]
        L.ctmhd_box_elems.restype = ctypes.c_int64
        L.ctmhd_workspace_bytes.argtypes = [_P, _B, ctypes.c_int]
        L.ctmhd_workspace_bytes.restype = ctypes.c_size_t
        L.ctmhd_step.argtypes = [_P, _B, _PTR5, _PTR3, ctypes.c_int, _vp, _vp, _vp, _vp,
                                 ctypes.c_size_t, _vp]
        L.ctmhd_step.restype = ctypes.c_int
        L.ctmhd_step_batched.argtypes = [_P, ctypes.c_int, _B, _vp, _PTR5, _PTR3, ctypes.c_int,
                                         ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.ctmhd_batch_plan_bytes.argtypes = [_P, _B, ctypes.c_int]
        L.ctmhd_batch_plan_bytes.restype = ctypes.c_size_t
        L.ctmhd_batch_plan.argtypes = [_P, _B, ctypes.c_int, _vp, ctypes.c_size_t]
        L.ctmhd_batch_plan.restype = ctypes.c_int
        L.ctmhd_step_batched.restype = ctypes.c_int
        _I3 = ctypes.POINTER(ctypes.c_int32)
        L.ctmhd_level_plan_bytes.argtypes = [_P, _B, _I3, ctypes.c_int, _I3]
        L.ctmhd_level_plan_bytes.restype = ctypes.c_size_t
        L.ctmhd_level_plan.argtypes = [_P, _B, _I3, ctypes.c_int, _I3, _vp, ctypes.c_size_t]
        L.ctmhd_level_plan.restype = ctypes.c_int
        L.ctmhd_step_level.argtypes = [_P, ctypes.c_int, _B, _I3, _I3, _vp, _PTR5, _PTR3,
                                       ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.ctmhd_step_level.restype = ctypes.c_int
        L.ctmhd_step_adjoint.argtypes = [_P, _B, _PTR5, _PTR3, _vp, _PTR5, _PTR3, _PTR5, _PTR3,
                                         _vp, ctypes.c_size_t, _vp]
        L.ctmhd_step_adjoint.restype = ctypes.c_int
        L.ctmhd_tape_bytes.argtypes = [_P, _B]
        L.ctmhd_tape_bytes.restype = ctypes.c_size_t
        L.ctmhd_step_record.argtypes = [_P, _B, _PTR5, _PTR3, _vp, _vp, ctypes.c_size_t, _vp,
                                        ctypes.c_size_t, _vp]
        L.ctmhd_step_record.restype = ctypes.c_int
        L.ctmhd_step_adjoint_tape.argtypes = [_P, _B, _vp, ctypes.c_size_t, _PTR5, _PTR3, _PTR5,
                                              _PTR3, _vp, ctypes.c_size_t, _vp]
        L.ctmhd_step_adjoint_tape.restype = ctypes.c_int
        L.ctmhd_adjoint_workspace_bytes.argtypes = [_P, _B]
        L.ctmhd_adjoint_workspace_bytes.restype = ctypes.c_size_t
        L.ctmhd_noalloc_scratch_bytes.argtypes = []
        L.ctmhd_noalloc_scratch_bytes.restype = ctypes.c_size_t
        L.ctmhd_step_noalloc.argtypes = [_P, _B, _PTR5, _PTR3, ctypes.c_int, _vp, _vp, _vp, _vp]
        L.ctmhd_step_noalloc.restype = ctypes.c_int
        L.ctmhd_profile_events.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
        L.ctmhd_profile_events.restype = ctypes.c_int
        L.ctmhd_profile_recorded.argtypes = []
        L.ctmhd_profile_recorded.restype = ctypes.c_int
        L.ctmhd_last_error.argtypes = []
        L.ctmhd_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


EXPORTED = ("ctmhd_required_ghosts", "ctmhd_box_elems", "ctmhd_workspace_bytes", "ctmhd_step",
            "ctmhd_batch_plan_bytes", "ctmhd_batch_plan", "ctmhd_step_batched",
            "ctmhd_level_plan_bytes", "ctmhd_level_plan", "ctmhd_step_level",
            "ctmhd_step_adjoint", "ctmhd_tape_bytes", "ctmhd_step_record",
            "ctmhd_step_adjoint_tape", "ctmhd_adjoint_workspace_bytes", "ctmhd_profile_events",
            "ctmhd_profile_recorded", "ctmhd_last_error", "ctmhd_noalloc_scratch_bytes",
            "ctmhd_step_noalloc")


def _check(rc):
    if rc != 0:
        raise CtmhdError(f"libctmhd error {rc}: {lib().ctmhd_last_error().decode()}")
    return rc


def make_params(gamma=5.0 / 3.0, eta=0.0, cfl=0.3, recon="plm", riemann="hlld", emf="q26",
                fofc=True, flag_mask=7, precision="fp64", force_flags=None, tile=0) -> Params:
    ff = None
    if force_flags is not None:
        ff = force_flags.data_ptr()
    return Params(float(gamma), float(eta), float(cfl), RECON[recon], RIEMANN[riemann], EMF[emf],
                  0, int(bool(fofc)), int(flag_mask), PRECISION[precision], int(tile), ff)


XCD_MAP = {"auto": 0, "contiguous": 1, "banded": 2}
EMF_KERNEL = {"auto": 0, "edge": 1, "march": 2}


def make_tile(chunk=0, strips=0, persistent=False, xrows=0, xcd_map="auto", emf_kernel="auto"):
    """The ctmhd_params.tile knob: minimum marching chunk, batched strips per
    work item, the batched schedule (per-phase launches or one persistent
    launch per step), the XCD mapping of the single-box edge and update
    passes ("auto", "contiguous": each XCD a contiguous range of tiles,
    "banded": all XCDs on bands of the same plane), the single-box Q26 edge
    kernel ("auto", "edge": one thread per edge position, "march": one thread
    per column of edges marching along z) and the x-face row segments per
    wavefront (0: defaults)."""
    return ((int(chunk) & 0xFF) | ((int(strips) & 0xFF) << 8) | ((1 if persistent else 0) << 16)
            | (XCD_MAP[xcd_map] << 19) | (EMF_KERNEL[emf_kernel] << 21)
            | ((int(xrows) & 0x7F) << 24))


def make_box(n, ng, dx, offset=0) -> Box:
    return Box((ctypes.c_int32 * 3)(*[int(v) for v in n]), int(ng),
               (ctypes.c_double * 3)(*[float(v) for v in dx]), int(offset))


def required_ghosts(params: Params) -> int:
    r = lib().ctmhd_required_ghosts(ctypes.byref(params))
    if r < 0:
        _check(r)
    return r


def workspace_bytes(params: Params, boxes) -> int:
    if isinstance(boxes, Box):
        boxes = [boxes]
    arr = (Box * len(boxes))(*boxes)
    return int(lib().ctmhd_workspace_bytes(ctypes.byref(params), arr, len(boxes)))


def _p(t):
    return None if t is None else t.data_ptr()


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def ctmhd_step(params: Params, box: Box, cons, bface, nsteps, dt_fixed=None, dt_out=None,
               diag=None, workspace=None, stream=None):
    """Direct binding of ctmhd_step; tensors are device tensors (float64 /
    int64 / uint8 workspace)."""
    ws = workspace
    rc = lib().ctmhd_step(ctypes.byref(params), ctypes.byref(box),
                          _PTR5(*[_p(t) for t in cons]), _PTR3(*[_p(t) for t in bface]),
                          int(nsteps), _p(dt_fixed), _p(dt_out), _p(diag), _p(ws),
                          ws.numel() if ws is not None else 0, _stream(stream))
    return _check(rc)


def noalloc_scratch_bytes() -> int:
    return int(lib().ctmhd_noalloc_scratch_bytes())


def ctmhd_step_noalloc(params: Params, box: Box, cons, bface, nsteps, dt_fixed=None,
                       dt_out=None, diag=None, stream=None):
    """Direct binding of ctmhd_step_noalloc (ctmhd_step on the library's fixed
    per-GPU scratch array instead of a caller workspace)."""
    rc = lib().ctmhd_step_noalloc(ctypes.byref(params), ctypes.byref(box),
                                  _PTR5(*[_p(t) for t in cons]), _PTR3(*[_p(t) for t in bface]),
                                  int(nsteps), _p(dt_fixed), _p(dt_out), _p(diag),
                                  _stream(stream))
    return _check(rc)


def batch_plan(params: Params, boxes):
    """Host plan bytes of the batched work queue (a numpy uint8 array)."""
    arr = (Box * len(boxes))(*boxes)
    n = int(lib().ctmhd_batch_plan_bytes(ctypes.byref(params), arr, len(boxes)))
    if n == 0:
        _check(-1)
    buf = np.zeros(n, np.uint8)
    _check(lib().ctmhd_batch_plan(ctypes.byref(params), arr, len(boxes),
                                  buf.ctypes.data_as(ctypes.c_void_p), n))
    return buf


def ctmhd_step_batched(params: Params, boxes, plan, cons, bface, nsteps, dt_mode=DT_GLOBAL,
                       dt_fixed=None, dt_out=None, diag=None, workspace=None, stream=None):
    arr = (Box * len(boxes))(*boxes)
    ws = workspace
    rc = lib().ctmhd_step_batched(ctypes.byref(params), len(boxes), arr, _p(plan),
                                  _PTR5(*[_p(t) for t in cons]), _PTR3(*[_p(t) for t in bface]),
                                  int(nsteps), int(dt_mode), _p(dt_fixed), _p(dt_out), _p(diag),
                                  _p(ws), ws.numel() if ws is not None else 0, _stream(stream))
    return _check(rc)


def _i32(v, n):
    arr = (ctypes.c_int32 * n)(*[int(x) for x in np.asarray(v).reshape(-1)])
    return arr


def level_plan(params: Params, boxes, origin, domain):
    """Host plan bytes of a level (boxes tiling the periodic domain; origin:
    (nbox, 3) level index of each box's first cell, axis 0 first)."""
    arr = (Box * len(boxes))(*boxes)
    org = _i32(origin, 3 * len(boxes))
    dom = _i32(domain, 3)
    n = int(lib().ctmhd_level_plan_bytes(ctypes.byref(params), arr, org, len(boxes), dom))
    if n == 0:
        raise CtmhdError("level plan size query failed (bad parameters, or the boxes do not "
                         "tile the domain)")
    buf = np.zeros(n, np.uint8)
    _check(lib().ctmhd_level_plan(ctypes.byref(params), arr, org, len(boxes), dom,
                                  buf.ctypes.data_as(ctypes.c_void_p), n))
    return buf


def ctmhd_step_level(params: Params, boxes, origin, domain, plan, cons, bface, nsteps,
                     dt_fixed=None, dt_out=None, diag=None, workspace=None, stream=None):
    arr = (Box * len(boxes))(*boxes)
    ws = workspace
    rc = lib().ctmhd_step_level(ctypes.byref(params), len(boxes), arr, _i32(origin, 3 * len(boxes)),
                                _i32(domain, 3), _p(plan), _PTR5(*[_p(t) for t in cons]),
                                _PTR3(*[_p(t) for t in bface]), int(nsteps), _p(dt_fixed),
                                _p(dt_out), _p(diag), _p(ws), ws.numel() if ws is not None else 0,
                                _stream(stream))
    return _check(rc)


def adjoint_workspace_bytes(params: Params, box: Box) -> int:
    return int(lib().ctmhd_adjoint_workspace_bytes(ctypes.byref(params), ctypes.byref(box)))


def ctmhd_step_adjoint(params: Params, box: Box, cons_n, bface_n, dt, g_cons, g_bface,
                       g_cons_out, g_bface_out, workspace=None, stream=None):
    ws = workspace
    rc = lib().ctmhd_step_adjoint(ctypes.byref(params), ctypes.byref(box),
                                  _PTR5(*[_p(t) for t in cons_n]), _PTR3(*[_p(t) for t in bface_n]),
                                  _p(dt), _PTR5(*[_p(t) for t in g_cons]),
                                  _PTR3(*[_p(t) for t in g_bface]),
                                  _PTR5(*[_p(t) for t in g_cons_out]),
                                  _PTR3(*[_p(t) for t in g_bface_out]), _p(ws),
                                  ws.numel() if ws is not None else 0, _stream(stream))
    return _check(rc)


def tape_bytes(params: Params, box: Box) -> int:
    return int(lib().ctmhd_tape_bytes(ctypes.byref(params), ctypes.byref(box)))


def ctmhd_step_record(params: Params, box: Box, cons, bface, dt, tape, workspace, stream=None):
    rc = lib().ctmhd_step_record(ctypes.byref(params), ctypes.byref(box),
                                 _PTR5(*[_p(t) for t in cons]), _PTR3(*[_p(t) for t in bface]),
                                 _p(dt), _p(tape), tape.numel(), _p(workspace), workspace.numel(),
                                 _stream(stream))
    return _check(rc)


def ctmhd_step_adjoint_tape(params: Params, box: Box, tape, g_cons, g_bface, g_cons_out,
                            g_bface_out, workspace, stream=None):
    rc = lib().ctmhd_step_adjoint_tape(ctypes.byref(params), ctypes.byref(box), _p(tape),
                                       tape.numel(), _PTR5(*[_p(t) for t in g_cons]),
                                       _PTR3(*[_p(t) for t in g_bface]),
                                       _PTR5(*[_p(t) for t in g_cons_out]),
                                       _PTR3(*[_p(t) for t in g_bface_out]), _p(workspace),
                                       workspace.numel(), _stream(stream))
    return _check(rc)


# ---------------------------------------------------------------------------
# Device state of one box and convenience wrappers.
# ---------------------------------------------------------------------------
class BoxState:
    """The 8 float64 fields of one ghosted box as device tensors."""

    def __init__(self, n, ng, dx, device="cuda"):
        import torch
        self.n = tuple(int(v) for v in n)
        self.ng = int(ng)
        self.dx = tuple(float(v) for v in dx)
        shape = tuple(v + 2 * self.ng for v in self.n[::-1])
        self.cons = [torch.zeros(shape, dtype=torch.float64, device=device) for _ in range(5)]
        self.bface = [torch.zeros(shape, dtype=torch.float64, device=device) for _ in range(3)]
        self.box = make_box(self.n, self.ng, self.dx)

    @classmethod
    def from_numpy(cls, cons, bface, ng, dx, device="cuda"):
        """Interior arrays (5|3, n2, n1, n0) -> ghosted device box (ghosts are
        filled by the library at the start of each step)."""
        import torch
        n2, n1, n0 = cons.shape[1:]
        st = cls((n0, n1, n2), ng, dx, device)
        g = st.ng
        sl = (slice(g, g + n2), slice(g, g + n1), slice(g, g + n0))
        for m in range(5):
            st.cons[m][sl] = torch.from_numpy(np.ascontiguousarray(cons[m])).to(device)
        for a in range(3):
            st.bface[a][sl] = torch.from_numpy(np.ascontiguousarray(bface[a])).to(device)
        return st

    def interior(self):
        g = self.ng
        n0, n1, n2 = self.n
        return (slice(g, g + n2), slice(g, g + n1), slice(g, g + n0))

    def to_numpy(self):
        sl = self.interior()
        c = np.stack([t[sl].cpu().numpy() for t in self.cons])
        b = np.stack([t[sl].cpu().numpy() for t in self.bface])
        return c, b


class Stepper:
    """Holds the workspace for one box and one parameter set."""

    def __init__(self, params: Params, state: BoxState):
        import torch
        self.params = params
        self.state = state
        nbytes = workspace_bytes(params, state.box)
        if nbytes == 0:
            raise CtmhdError("workspace size query failed")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=state.cons[0].device)
        if self.workspace.data_ptr() % 256:
            raise CtmhdError("workspace allocation is not 256-byte aligned")

    def step(self, nsteps=1, dt_fixed=None, dt_out=None, diag=None, stream=None):
        ctmhd_step(self.params, self.state.box, self.state.cons, self.state.bface, nsteps,
                   dt_fixed, dt_out, diag, self.workspace, stream)


def run(params: Params, cons, bface, dx, nsteps=1, dt_fixed=None, ng=None, device="cuda"):
    """Convenience: numpy interior state in, numpy interior state out, with
    the per-step dt values and diagnostics."""
    import torch
    if ng is None:
        ng = required_ghosts(params)
    st = BoxState.from_numpy(cons, bface, ng, dx, device)
    S = Stepper(params, st)
    dts = torch.zeros(nsteps, dtype=torch.float64, device=device)
    diag = torch.zeros(4 * nsteps, dtype=torch.int64, device=device)
    dtf = None
    if dt_fixed is not None:
        dtf = torch.as_tensor(np.broadcast_to(np.asarray(dt_fixed, np.float64), (nsteps,)).copy(),
                              device=device)
    S.step(nsteps, dtf, dts, diag)
    torch.cuda.synchronize()
    c, b = st.to_numpy()
    return c, b, dts.cpu().numpy(), diag.cpu().numpy().reshape(nsteps, 4)


# ---------------------------------------------------------------------------
# HIP event timing of the library's face kernel (benchmarks).
# ---------------------------------------------------------------------------
class KernelTimer:
    """Creates HIP events through the HIP runtime and hands them to
    ctmhd_profile_events; mean_ms() gives the average duration of the
    recorded face-kernel launches (after a synchronisation)."""

    def __init__(self, npairs):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.events = (ctypes.c_void_p * (2 * npairs))()
        for i in range(2 * npairs):
            ev = ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(ev)) != 0:
                raise CtmhdError("hipEventCreate failed")
            self.events[i] = ev
        self.npairs = npairs

    def start(self):
        _check(lib().ctmhd_profile_events(self.events, self.npairs))

    def stop(self):
        n = lib().ctmhd_profile_recorded()
        _check(lib().ctmhd_profile_events(None, 0))
        return n

    def durations_ms(self, n):
        out = []
        for i in range(n):
            ms = ctypes.c_float()
            rc = self.hip.hipEventElapsedTime(ctypes.byref(ms), self.events[2 * i],
                                              self.events[2 * i + 1])
            if rc != 0:
                raise CtmhdError(f"hipEventElapsedTime failed ({rc})")
            out.append(ms.value)
        return out

    def close(self):
        for i in range(2 * self.npairs):
            self.hip.hipEventDestroy(self.events[i])


# ---------------------------------------------------------------------------
# Batched boxes: packed device arrays and convenience wrappers.
# ---------------------------------------------------------------------------
class BatchedState:
    """Many ghosted boxes packed back to back in 8 float64 device arrays."""

    def __init__(self, shapes, ng, dxs, device="cuda"):
        import torch
        self.ng = int(ng)
        self.shapes = [tuple(int(v) for v in n) for n in shapes]
        self.dxs = [tuple(float(v) for v in dx) for dx in dxs]
        self.offsets = []
        off = 0
        self.boxes = []
        for n, dx in zip(self.shapes, self.dxs):
            self.offsets.append(off)
            self.boxes.append(make_box(n, self.ng, dx, off))
            off += (n[0] + 2 * ng) * (n[1] + 2 * ng) * (n[2] + 2 * ng)
        self.total = off
        self.cons = [torch.zeros(off, dtype=torch.float64, device=device) for _ in range(5)]
        self.bface = [torch.zeros(off, dtype=torch.float64, device=device) for _ in range(3)]

    def _view(self, t, b):
        n = self.shapes[b]
        g = self.ng
        e = (n[0] + 2 * g) * (n[1] + 2 * g) * (n[2] + 2 * g)
        return t[self.offsets[b]:self.offsets[b] + e].view(n[2] + 2 * g, n[1] + 2 * g, n[0] + 2 * g)

    def _interior(self, b):
        g = self.ng
        n = self.shapes[b]
        return (slice(g, g + n[2]), slice(g, g + n[1]), slice(g, g + n[0]))

    @classmethod
    def from_numpy(cls, states, ng, device="cuda"):
        """states: list of (cons (5,n2,n1,n0), bface (3,n2,n1,n0), dx)."""
        import torch
        shapes = [(c.shape[3], c.shape[2], c.shape[1]) for c, _, _ in states]
        st = cls(shapes, ng, [dx for _, _, dx in states], device)
        # fill on the host, one transfer per field
        hc = [np.zeros(st.total) for _ in range(5)]
        hb = [np.zeros(st.total) for _ in range(3)]
        for b, (c, bf, _) in enumerate(states):
            n = st.shapes[b]
            g = st.ng
            shp = (n[2] + 2 * g, n[1] + 2 * g, n[0] + 2 * g)
            sl = st._interior(b)
            e = shp[0] * shp[1] * shp[2]
            for m in range(5):
                hc[m][st.offsets[b]:st.offsets[b] + e].reshape(shp)[sl] = c[m]
            for a in range(3):
                hb[a][st.offsets[b]:st.offsets[b] + e].reshape(shp)[sl] = bf[a]
        for m in range(5):
            st.cons[m].copy_(torch.from_numpy(hc[m]))
        for a in range(3):
            st.bface[a].copy_(torch.from_numpy(hb[a]))
        return st

    def to_numpy(self):
        hc = [t.cpu().numpy() for t in self.cons]
        hb = [t.cpu().numpy() for t in self.bface]
        out = []
        for b in range(len(self.shapes)):
            n = self.shapes[b]
            g = self.ng
            shp = (n[2] + 2 * g, n[1] + 2 * g, n[0] + 2 * g)
            e = shp[0] * shp[1] * shp[2]
            sl = self._interior(b)
            c = np.stack([hc[m][self.offsets[b]:self.offsets[b] + e].reshape(shp)[sl] for m in range(5)])
            bf = np.stack([hb[a][self.offsets[b]:self.offsets[b] + e].reshape(shp)[sl] for a in range(3)])
            out.append((c, bf))
        return out


class BatchedStepper:
    """Workspace and device plan for one parameter set and one set of boxes."""

    def __init__(self, params: Params, state: BatchedState):
        import torch
        self.params = params
        self.state = state
        dev = state.cons[0].device
        plan = batch_plan(params, state.boxes)
        self.plan = torch.from_numpy(plan).to(dev)
        nbytes = workspace_bytes(params, state.boxes)
        if nbytes == 0:
            raise CtmhdError("workspace size query failed")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        if self.workspace.data_ptr() % 256 or self.plan.data_ptr() % 16:
            raise CtmhdError("workspace / plan allocation is not aligned")

    def step(self, nsteps=1, dt_mode=DT_GLOBAL, dt_fixed=None, dt_out=None, diag=None,
             stream=None):
        ctmhd_step_batched(self.params, self.state.boxes, self.plan, self.state.cons,
                           self.state.bface, nsteps, dt_mode, dt_fixed, dt_out, diag,
                           self.workspace, stream)


def run_batched(params: Params, states, nsteps=1, dt_mode=DT_GLOBAL, dt_fixed=None, ng=None,
                device="cuda"):
    """Convenience: list of numpy (cons, bface, dx) in, list of (cons, bface)
    out, with dt values (nsteps or nsteps x nbox) and per-step diagnostics."""
    import torch
    if ng is None:
        ng = required_ghosts(params)
    st = BatchedState.from_numpy(states, ng, device)
    S = BatchedStepper(params, st)
    ndt = len(states) if dt_mode == DT_PER_BOX else 1
    dts = torch.zeros(nsteps * ndt, dtype=torch.float64, device=device)
    diag = torch.zeros(4 * nsteps, dtype=torch.int64, device=device)
    dtf = None
    if dt_fixed is not None:
        dtf = torch.as_tensor(np.asarray(dt_fixed, np.float64).reshape(-1).copy(), device=device)
    S.step(nsteps, dt_mode, dtf, dts, diag)
    torch.cuda.synchronize()
    return st.to_numpy(), dts.cpu().numpy().reshape(nsteps, ndt), diag.cpu().numpy().reshape(nsteps, 4)


# ---------------------------------------------------------------------------
# A level: boxes that tile one periodic domain, ghosts exchanged between them.
# ---------------------------------------------------------------------------
class LevelStepper:
    """Workspace and device plan of a level over the packed boxes of `state`."""

    def __init__(self, params: Params, state: BatchedState, origin, domain):
        import torch
        self.params = params
        self.state = state
        self.origin = np.asarray(origin, np.int32).reshape(len(state.boxes), 3)
        self.domain = tuple(int(v) for v in domain)
        dev = state.cons[0].device
        self.plan = torch.from_numpy(level_plan(params, state.boxes, self.origin, self.domain)).to(dev)
        nbytes = workspace_bytes(params, state.boxes)
        if nbytes == 0:
            raise CtmhdError("workspace size query failed")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        if self.workspace.data_ptr() % 256 or self.plan.data_ptr() % 16:
            raise CtmhdError("workspace / plan allocation is not aligned")

    def step(self, nsteps=1, dt_fixed=None, dt_out=None, diag=None, stream=None):
        ctmhd_step_level(self.params, self.state.boxes, self.origin, self.domain, self.plan,
                         self.state.cons, self.state.bface, nsteps, dt_fixed, dt_out, diag,
                         self.workspace, stream)


def split_level(cons, bface, dx, cuts, shift=(0, 0, 0)):
    """Cut a periodic domain (numpy cons (5, n2, n1, n0), bface (3, ...)) into
    boxes: cuts[d] are the increasing box boundaries along axis d (0 ... n_d),
    and every box starts `shift` cells further along (wrapping), so that boxes
    may straddle the periodic boundary.  Returns [(cons, bface, dx)], origin."""
    n = (cons.shape[3], cons.shape[2], cons.shape[1])
    states, origin = [], []
    for k in range(len(cuts[2]) - 1):
        for j in range(len(cuts[1]) - 1):
            for i in range(len(cuts[0]) - 1):
                lo = [cuts[0][i], cuts[1][j], cuts[2][k]]
                hi = [cuts[0][i + 1], cuts[1][j + 1], cuts[2][k + 1]]
                o = [(lo[d] + shift[d]) % n[d] for d in range(3)]
                idx = [np.arange(o[d], o[d] + hi[d] - lo[d]) % n[d] for d in range(3)]
                sel = np.ix_(idx[2], idx[1], idx[0])
                c = np.stack([cons[m][sel] for m in range(5)])
                b = np.stack([bface[a][sel] for a in range(3)])
                states.append((c, b, tuple(dx)))
                origin.append(o)
    return states, np.asarray(origin, np.int32)


def join_level(parts, origin, domain):
    """Inverse of split_level: list of (cons, bface) boxes -> domain arrays."""
    n0, n1, n2 = domain
    cons = np.zeros((5, n2, n1, n0))
    bface = np.zeros((3, n2, n1, n0))
    for (c, b), o in zip(parts, origin):
        m = (c.shape[3], c.shape[2], c.shape[1])
        idx = [np.arange(o[d], o[d] + m[d]) % domain[d] for d in range(3)]
        sel = np.ix_(idx[2], idx[1], idx[0])
        for q in range(5):
            cons[q][sel] = c[q]
        for a in range(3):
            bface[a][sel] = b[a]
    return cons, bface


def run_level(params: Params, cons, bface, dx, cuts, nsteps=1, dt_fixed=None, shift=(0, 0, 0),
              ng=None, device="cuda"):
    """Convenience: cut the domain into a level of boxes, advance it with
    ctmhd_step_level and join the result.  Returns (cons, bface, dts, diag)."""
    import torch
    if ng is None:
        ng = required_ghosts(params)
    states, origin = split_level(cons, bface, dx, cuts, shift)
    domain = (cons.shape[3], cons.shape[2], cons.shape[1])
    st = BatchedState.from_numpy(states, ng, device)
    S = LevelStepper(params, st, origin, domain)
    dts = torch.zeros(nsteps, dtype=torch.float64, device=device)
    diag = torch.zeros(4 * nsteps, dtype=torch.int64, device=device)
    dtf = None
    if dt_fixed is not None:
        dtf = torch.as_tensor(np.asarray(dt_fixed, np.float64).reshape(-1).copy(), device=device)
    S.step(nsteps, dtf, dts, diag)
    torch.cuda.synchronize()
    c, b = join_level(st.to_numpy(), origin, domain)
    return c, b, dts.cpu().numpy(), diag.cpu().numpy().reshape(nsteps, 4)


def parse_plan(plan):
    """Decode a host plan (for checks on the CPU): header fields, box order,
    per-phase item prefixes."""
    import struct
    buf = bytes(plan)
    nbox, nphase, strips, magic = struct.unpack_from("4i", buf, 0)
    (key,) = struct.unpack_from("Q", buf, 16)
    kmax = 24
    o = 24
    kind = list(struct.unpack_from(f"{kmax}i", buf, o)); o += 4 * kmax
    stage = list(struct.unpack_from(f"{kmax}i", buf, o)); o += 4 * kmax
    item_off = list(struct.unpack_from(f"{kmax}i", buf, o)); o += 4 * kmax
    rng = struct.unpack_from("6i", buf, o); o += 24
    range_items = struct.unpack_from("3i", buf, o); o += 12
    o = (o + 7) & ~7
    order_off, prefix_off, desc_off = struct.unpack_from("3q", buf, o); o += 24
    xarg = list(struct.unpack_from(f"{kmax}i", buf, o)); o += 4 * kmax
    level, nxblk = struct.unpack_from("2i", buf, o); o += 8
    xbox_off, xblk_off = struct.unpack_from("2q", buf, o)
    order = np.frombuffer(buf, np.int32, nbox, order_off)
    xbox = xblk = None
    if level:
        xbox = np.frombuffer(buf, np.int32, nbox + 1, xbox_off)
        xblk = np.frombuffer(buf, np.dtype([("dst", "<i8"), ("src", "<i8"), ("dsy", "<i4"),
                                            ("dsz", "<i4"), ("ssy", "<i4"), ("ssz", "<i4"),
                                            ("ex", "<i4"), ("ey", "<i4"), ("vol_lo", "<i4"),
                                            ("vol", "<i4")]), nxblk, xblk_off)
    prefix = np.frombuffer(buf, np.int32, nphase * (nbox + 1), prefix_off).reshape(nphase, nbox + 1)
    return dict(nbox=nbox, nphase=nphase, strips=strips, magic=magic, key=key, kind=kind[:nphase],
                stage=stage[:nphase], item_off=item_off[:nphase],
                range=[rng[0:2], rng[2:4], rng[4:6]], range_items=list(range_items),
                order=order, prefix=prefix, xarg=xarg[:nphase], level=level, xbox=xbox, xblk=xblk)
