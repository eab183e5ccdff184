"""Python binding of libhsma (argument marshalling only).

Every step of the HSMA update step runs in the library's HIP kernels; this
module converts arguments, owns device buffers through PyTorch (device memory
and streams only) and raises on every non-OK status.  Names follow the C ABI
in include/hsma.h.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libhsma.so")

BC_PERIODIC = 0
BC_METALLIC = 1
BC_SLAB = 2
BC_DIELECTRIC = 3
FP64 = 0
FP32_COMP = 1
NEAR_BLOCK = 0
NEAR_SPHERE = 1
NEAR_TREE = 2
DIPOLE_EXACT = 0
DIPOLE_LAYERS = 1
FAR_SURFACE = 0
FAR_DIRECT = 1
DTYPE_F64 = 0     # element type of the arrays of hsma_energy_forces_device_typed
DTYPE_F32 = 1
DEFAULT_SEED = 12345

_lib = None


class HsmaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("HSMA status %d: %s" % (status, msg))
        self.status = status


class PlanDesc(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("bc", ctypes.c_int), ("p", ctypes.c_int),
                ("M", ctypes.c_int), ("K", ctypes.c_int), ("R", ctypes.c_double),
                ("precision", ctypes.c_int), ("seed", ctypes.c_uint64), ("near_mode", ctypes.c_int),
                ("dipole_mode", ctypes.c_int), ("dr", ctypes.c_double), ("far_mode", ctypes.c_int),
                ("gamma", ctypes.c_double), ("far_shells", ctypes.c_int), ("tree_order", ctypes.c_int),
                ("tree_min_n", ctypes.c_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_basis", ctypes.c_int), ("n_unknowns", ctypes.c_int), ("K", ctypes.c_int),
                ("n_check", ctypes.c_int), ("M_eff", ctypes.c_int), ("F1", ctypes.c_int),
                ("F2", ctypes.c_int), ("R0", ctypes.c_double), ("Rs", ctypes.c_double),
                ("precision", ctypes.c_int), ("bc", ctypes.c_int),
                ("bytes_resident", ctypes.c_size_t), ("near_mode", ctypes.c_int),
                ("max_images_per_source", ctypes.c_int), ("dipole_mode", ctypes.c_int),
                ("dr", ctypes.c_double), ("far_mode", ctypes.c_int), ("gamma", ctypes.c_double),
                ("far_shells", ctypes.c_int), ("tree_order", ctypes.c_int), ("tree_min_n", ctypes.c_int)]


class Intermediates(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("b", "A", "surf", "phi_near", "field_near", "phi_out", "field_out")]


class ServerDesc(ctypes.Structure):
    _fields_ = [("memory_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int),
                ("precision", ctypes.c_int), ("refine_below", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("active", ctypes.c_int), ("pending", ctypes.c_int),
                ("ticks", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("arena_bytes", ctypes.c_size_t), ("arena_used", ctypes.c_size_t),
                ("arena_peak", ctypes.c_size_t), ("refined", ctypes.c_int64)]


class NearSchedule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("rows_per_lane", ctypes.c_int), ("block", ctypes.c_int),
                ("slices", ctypes.c_int), ("parts", ctypes.c_int), ("blocks", ctypes.c_int),
                ("launches", ctypes.c_int)]


_TRACE_ARGS = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]

EXPORTS = {
    "hsma_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "hsma_last_error": (ctypes.c_char_p, []),
    "hsma_version": (ctypes.c_int, []),
    "hsma_plan_create": (ctypes.c_int, [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_void_p)]),
    "hsma_plan_create_ex": (ctypes.c_int, [ctypes.POINTER(PlanDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "hsma_plan_destroy": (None, [ctypes.c_void_p]),
    "hsma_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PlanInfo)]),
    "hsma_plan_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "hsma_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int64]),
    "hsma_near_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(NearSchedule)]),
    "hsma_energy_forces": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "hsma_energy_forces_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_size_t, ctypes.POINTER(ctypes.c_double),
                                                 ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.POINTER(Intermediates)]),
    "hsma_energy_forces_device_typed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                       ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                                       ctypes.c_void_p, ctypes.c_size_t,
                                                       ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                                       ctypes.c_void_p]),
    "hsma_energy_forces_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_int64, ctypes.c_void_p,
                                                  ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                                  ctypes.c_void_p]),
    "hsma_energy_grad_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_size_t, ctypes.POINTER(ctypes.c_double),
                                               ctypes.c_void_p, ctypes.c_void_p]),
    "hsma_server_create": (ctypes.c_int, [ctypes.POINTER(ServerDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "hsma_server_destroy": (None, [ctypes.c_void_p]),
    "hsma_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "hsma_server_tick": (ctypes.c_int, [ctypes.c_void_p]),
    "hsma_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "hsma_server_result": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "hsma_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "hsma_server_run_trace": (ctypes.c_int, [ctypes.c_void_p] + _TRACE_ARGS),
    "hsma_run_trace_sequential": (ctypes.c_int, _TRACE_ARGS),
    "hsma_timing_enable": (ctypes.c_int, [ctypes.c_int]),
    "hsma_timing_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
}


def load():
    """Load libhsma.so; raise if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhsma.so not built: run paper_1806_04801_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(st):
    if st != 0:
        lib = load()
        raise HsmaError(st, "%s: %s" % (lib.hsma_status_string(st).decode(),
                                        lib.hsma_last_error().decode()))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_handle(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """An HSMA plan (preparation step) resident on the current GPU."""

    def __init__(self, L, bc, p, M, K, R, precision=FP64, seed=DEFAULT_SEED, near_mode=NEAR_BLOCK,
                 dipole_mode=DIPOLE_EXACT, dr=0.0, far_mode=FAR_SURFACE, gamma=0.0, far_shells=0,
                 tree_order=0, tree_min_n=0):
        lib = load()
        d = PlanDesc(L=float(L), bc=int(bc), p=int(p), M=int(M), K=int(K), R=float(R),
                     precision=int(precision), seed=int(seed), near_mode=int(near_mode),
                     dipole_mode=int(dipole_mode), dr=float(dr), far_mode=int(far_mode),
                     gamma=float(gamma), far_shells=int(far_shells), tree_order=int(tree_order),
                     tree_min_n=int(tree_min_n))
        h = ctypes.c_void_p()
        _check(lib.hsma_plan_create_ex(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.L, self.bc, self.p, self.M, self.K, self.R = float(L), int(bc), int(p), int(M), int(K), float(R)
        self.precision = int(precision)
        inf = PlanInfo()
        _check(lib.hsma_plan_info(h, ctypes.byref(inf)))
        self.info = {f: getattr(inf, f) for f, _ in PlanInfo._fields_}
        self._ws = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hsma_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def points(self, which):
        """Host copies of the plan geometry (centred): 0 monitoring points,
        1 twins, 2 surface points (returns (xyz, weights))."""
        n = self.info["M_eff"] if which == 2 else self.info["K"]
        xyz = np.zeros((n, 3))
        w = np.zeros(n) if which == 2 else None
        _check(load().hsma_plan_points(self._h, which, xyz.ctypes.data_as(ctypes.c_void_p),
                                       w.ctypes.data_as(ctypes.c_void_p) if w is not None else None))
        return (xyz, w) if which == 2 else xyz

    def workspace_bytes(self, n):
        return int(load().hsma_workspace_bytes(self._h, int(n)))

    def near_schedule(self, n):
        """The near-field kernel a step with n particles runs (see hsma.h):
        kind 0 per-target tiles, kind 1 each unordered pair once."""
        out = NearSchedule()
        _check(load().hsma_near_schedule(self._h, int(n), ctypes.byref(out)))
        return {f: getattr(out, f) for f, _ in NearSchedule._fields_}

    def workspace(self, n, device):
        import torch
        need = self.workspace_bytes(n)
        if self._ws is None or self._ws.numel() < need or self._ws.device != device:
            self._ws = torch.empty(need, dtype=torch.uint8, device=device)
        return self._ws

    # ------------------------------------------------------------ host path
    def energy_forces_host(self, x, q):
        """Host arrays in, host arrays out (the library copies over PCIe)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        q = np.ascontiguousarray(q, dtype=np.float64)
        n = len(q)
        e = ctypes.c_double()
        phi = np.zeros(n)
        F = np.zeros((n, 3))
        _check(load().hsma_energy_forces(self._h, x.ctypes.data_as(ctypes.c_void_p),
                                         q.ctypes.data_as(ctypes.c_void_p), n, ctypes.byref(e),
                                         phi.ctypes.data_as(ctypes.c_void_p),
                                         F.ctypes.data_as(ctypes.c_void_p)))
        return e.value, phi, F

    # ------------------------------------------------------------ device path
    def energy_forces(self, x, q, phi=None, forces=None, intermediates=False):
        """x (N x 3), q (N): CUDA tensors, both float64 or both float32 (phi
        and forces then come back in the same type).  Returns (energy, phi,
        forces) and, if intermediates (float64 only), a dict of the stage
        outputs."""
        import torch
        assert x.is_cuda and q.is_cuda and x.dtype == q.dtype
        assert x.dtype in (torch.float64, torch.float32)
        x = x.contiguous()
        q = q.contiguous()
        n = q.numel()
        dev = x.device
        if x.dtype == torch.float32:
            assert not intermediates, "intermediates need float64 inputs"
            if phi is None:
                phi = torch.empty(n, dtype=torch.float32, device=dev)
            if forces is None:
                forces = torch.empty((n, 3), dtype=torch.float32, device=dev)
            ws = self.workspace(n, dev)
            e = ctypes.c_double()
            _check(load().hsma_energy_forces_device_typed(
                self._h, _ptr(x), _ptr(q), n, DTYPE_F32, _stream_handle(torch, dev), _ptr(ws), ws.numel(),
                ctypes.byref(e), _ptr(phi), _ptr(forces)))
            return e.value, phi, forces
        if phi is None:
            phi = torch.empty(n, dtype=torch.float64, device=dev)
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=dev)
        ws = self.workspace(n, dev)
        dbg = None
        inter = None
        if intermediates:
            inter = {
                "b": torch.empty(self.info["K"], dtype=torch.float64, device=dev),
                "A": torch.empty(self.info["n_basis"], dtype=torch.float64, device=dev),
                "surf": torch.empty((self.info["M_eff"], 8), dtype=torch.float64, device=dev),
                "phi_near": torch.empty(n, dtype=torch.float64, device=dev),
                "field_near": torch.empty((n, 3), dtype=torch.float64, device=dev),
                "phi_out": torch.empty(n, dtype=torch.float64, device=dev),
                "field_out": torch.empty((n, 3), dtype=torch.float64, device=dev),
            }
            dbg = Intermediates(**{k: v.data_ptr() for k, v in inter.items()})
        e = ctypes.c_double()
        _check(load().hsma_energy_forces_device(
            self._h, _ptr(x), _ptr(q), n, _stream_handle(torch, dev), _ptr(ws), ws.numel(),
            ctypes.byref(e), _ptr(phi), _ptr(forces), ctypes.byref(dbg) if dbg is not None else None))
        if intermediates:
            return e.value, phi, forces, inter
        return e.value, phi, forces

    def energy_forces_noalloc(self, x, q, phi, forces):
        """The allocation-free entry point: x (N x 3), q (N), phi (N), forces
        (N x 3) float64 CUDA tensors allocated by the caller; the library runs
        in its static device scratch.  Returns the energy."""
        import torch
        for t in (x, q, phi, forces):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
        n = q.numel()
        assert x.numel() == 3 * n and phi.numel() == n and forces.numel() == 3 * n
        e = ctypes.c_double()
        _check(load().hsma_energy_forces_noalloc(self._h, _ptr(x), _ptr(q), n,
                                                 _stream_handle(torch, x.device), ctypes.byref(e),
                                                 _ptr(phi), _ptr(forces)))
        return e.value

    def energy_grad(self, x, q):
        """Exact gradient of the computed energy: (energy, dE/dx, dE/dq)."""
        import torch
        x = x.contiguous()
        q = q.contiguous()
        n = q.numel()
        dev = x.device
        dx = torch.empty((n, 3), dtype=torch.float64, device=dev)
        dq = torch.empty(n, dtype=torch.float64, device=dev)
        ws = self.workspace(n, dev)
        e = ctypes.c_double()
        _check(load().hsma_energy_grad_device(self._h, _ptr(x), _ptr(q), n, _stream_handle(torch, dev),
                                              _ptr(ws), ws.numel(), ctypes.byref(e), _ptr(dx), _ptr(dq)))
        return e.value, dx, dq


# Default double-precision refinement threshold of a single-precision server:
# an energy below this fraction of 1/2 sum |q_i phi_i| is recomputed in double
# precision (kept every energy of a 4096-request serving mix within 1e-5 of
# the double-precision result, refining about 2 % of the requests).
DEFAULT_REFINE_BELOW = 3e-3


class Server:
    """Continuous-batching server of energy/force requests (see hsma.h).
    refine_below=None selects DEFAULT_REFINE_BELOW for a single-precision
    server and 0 (off) for a double-precision one; the refinement also
    covers requests on the fast multipole method (tree plans)."""

    def __init__(self, memory_bytes=8 << 30, max_active=64, precision=FP32_COMP, refine_below=None):
        lib = load()
        if refine_below is None:
            refine_below = DEFAULT_REFINE_BELOW if int(precision) == FP32_COMP else 0.0
        d = ServerDesc(memory_bytes=int(memory_bytes), max_active=int(max_active),
                       precision=int(precision), refine_below=float(refine_below))
        h = ctypes.c_void_p()
        _check(lib.hsma_server_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._plans = []

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hsma_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, plan, x, q):
        x = np.ascontiguousarray(x, dtype=np.float64)
        q = np.ascontiguousarray(q, dtype=np.float64)
        rid = ctypes.c_int64()
        _check(load().hsma_server_submit(self._h, plan.handle, x.ctypes.data_as(ctypes.c_void_p),
                                         q.ctypes.data_as(ctypes.c_void_p), len(q), ctypes.byref(rid)))
        self._plans.append(plan)
        return rid.value

    def tick(self):
        _check(load().hsma_server_tick(self._h))

    def wait(self, rid):
        _check(load().hsma_server_wait(self._h, int(rid)))

    def result(self, rid, n):
        """(done, energy, phi, forces, latency_s); releases the request when done."""
        done = ctypes.c_int()
        e = ctypes.c_double()
        lat = ctypes.c_double()
        phi = np.zeros(n)
        F = np.zeros((n, 3))
        _check(load().hsma_server_result(self._h, int(rid), ctypes.byref(done), ctypes.byref(e),
                                         phi.ctypes.data_as(ctypes.c_void_p),
                                         F.ctypes.data_as(ctypes.c_void_p), ctypes.byref(lat)))
        if not done.value:
            return False, None, None, None, None
        return True, e.value, phi, F, lat.value

    def stats(self):
        st = ServerStats()
        _check(load().hsma_server_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def run_trace(self, arrivals, plans, xs, qs):
        return _trace(load().hsma_server_run_trace, [self._h], arrivals, plans, xs, qs)


def run_trace_sequential(arrivals, plans, xs, qs):
    """Open-loop replay with one plain solve per request (each plan's precision)."""
    return _trace(load().hsma_run_trace_sequential, [], arrivals, plans, xs, qs)


def _trace(fn, head, arrivals, plans, xs, qs):
    n = len(arrivals)
    arr = np.ascontiguousarray(arrivals, dtype=np.float64)
    xs = [np.ascontiguousarray(v, dtype=np.float64) for v in xs]
    qs = [np.ascontiguousarray(v, dtype=np.float64) for v in qs]
    ph = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    xp = (ctypes.c_void_p * n)(*[v.ctypes.data for v in xs])
    qp = (ctypes.c_void_p * n)(*[v.ctypes.data for v in qs])
    Ns = np.array([len(v) for v in qs], dtype=np.int64)
    en = np.zeros(n)
    lat = np.zeros(n)
    wall = ctypes.c_double()
    _check(fn(*head, n, arr.ctypes.data_as(ctypes.c_void_p), ctypes.cast(ph, ctypes.c_void_p),
              ctypes.cast(xp, ctypes.c_void_p), ctypes.cast(qp, ctypes.c_void_p),
              Ns.ctypes.data_as(ctypes.c_void_p), en.ctypes.data_as(ctypes.c_void_p),
              lat.ctypes.data_as(ctypes.c_void_p), ctypes.byref(wall)))
    return en, lat, wall.value


def timing_enable(flag=True):
    _check(load().hsma_timing_enable(1 if flag else 0))


def timing_read():
    ms = (ctypes.c_double * 3)()
    n = (ctypes.c_int64 * 3)()
    _check(load().hsma_timing_read(ms, n))
    return {"near": (ms[0], n[0]), "rhs": (ms[1], n[1]), "surface": (ms[2], n[2])}


def make_energy_function():
    """torch.autograd.Function whose forward returns the HSMA energy of (x, q)
    and whose backward applies the library's adjoint kernels."""
    import torch

    class HsmaEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, q, plan):
            e, dx, dq = plan.energy_grad(x.detach(), q.detach())
            ctx.save_for_backward(dx, dq)
            return torch.tensor(e, dtype=torch.float64, device=x.device)

        @staticmethod
        def backward(ctx, g):
            dx, dq = ctx.saved_tensors
            return g * dx, g * dq, None

    return HsmaEnergy
