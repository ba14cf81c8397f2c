"""Thin ctypes binding of libdghabc (include/dghabc.h).

Argument marshalling only: every step of the time stepper runs in the
library's HIP kernels.  PyTorch provides the device workspace (a uint8
tensor) and the stream.  The binding raises if the library is missing: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DGHABC_LIB may point at another build of the same library (e.g. a tuning
# variant); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("DGHABC_LIB", os.path.join(_HERE, "libdghabc.so"))

DGH_OK = 0
STATUS = {0: "DGH_OK", -1: "DGH_EINVAL", -2: "DGH_ESTATE", -3: "DGH_EHIP", -4: "DGH_ENOMEM",
          -5: "DGH_ENONFINITE", -6: "DGH_EUNSTABLE"}
BC = {"habc": 0, "abc": 1, "dirichlet": 2, "periodic": 3}
ARRAYS = ["q3", "res3", "q2", "res2", "qb3", "q0_3", "q1", "res1", "qb2", "q0_2", "qb1"]
COUNTS = ["K", "Ktri", "Klin", "Kpnt", "Np", "Np2", "Np1", "P", "N", "n_shots"]

# exported names and their C signatures
_SIGS = {
    "dgh_create": [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int],
    "dgh_upload_mesh": [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                        C.c_void_p],
    "dgh_set_order": [C.c_void_p, C.c_int],
    "dgh_set_habc": [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p],
    "dgh_set_material": [C.c_void_p, C.c_void_p, C.c_void_p],
    "dgh_counts": [C.c_void_p, C.c_void_p],
    "dgh_node_coords": [C.c_void_p, C.c_void_p],
    "dgh_workspace_size": [C.c_void_p, C.POINTER(C.c_size_t)],
    "dgh_bind_workspace": [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p],
    "dgh_set_state": [C.c_void_p, C.c_int, C.c_void_p],
    "dgh_read_fields": [C.c_void_p, C.c_int, C.c_void_p],
    "dgh_set_source": [C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_double, C.c_double],
    "dgh_step": [C.c_void_p, C.c_int, C.c_double, C.c_double],
    "dgh_set_graph": [C.c_void_p, C.c_int],
    "dgh_step_group": [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double],
    "dgh_tuning_count": [C.c_void_p, C.POINTER(C.c_int)],
    "dgh_set_tuning": [C.c_void_p, C.c_int],
    "dgh_autotune": [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.c_void_p],
    "dgh_energy": [C.c_void_p, C.c_int, C.POINTER(C.c_double)],
    "dgh_check": [C.c_void_p, C.c_int, C.c_double, C.c_double, C.POINTER(C.c_double)],
    "dgh_set_closure": [C.c_void_p, C.c_void_p, C.c_int],
    "dgh_closure_record": [C.c_void_p, C.c_int],
    "dgh_set_closure_memory": [C.c_void_p, C.c_void_p],
    "dgh_closure_sample": [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p],
    "dgh_mlp_work_size": [C.c_int, C.POINTER(C.c_size_t)],
    "dgh_mlp_forward": [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p],
    "dgh_mlp_grad": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                     C.POINTER(C.c_double), C.c_void_p],
    "dgh_mlp_adam": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_float,
                     C.c_void_p],
    "dgh_mlp_grad_bf16": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                          C.POINTER(C.c_double), C.c_void_p],
    "dgh_mlp_grad_static": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                            C.POINTER(C.c_double), C.c_void_p],
    "dgh_kernel_timing": [C.c_void_p, C.c_int],
    "dgh_kernel_time": [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_longlong)],
    "dgh_last_error": [C.c_void_p],
    "dgh_destroy": [C.c_void_p],
}

_lib = None


def load():
    """Loads the built library; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch first: its bundled HIP runtime has the same soname as the one
        # the library links, so both then share a single runtime instance
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        lib = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = C.c_char_p if name == "dgh_last_error" else (
                None if name == "dgh_destroy" else C.c_int)
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class DghError(RuntimeError):
    pass


class Solver:
    """One context of the library: mesh, order N, HABC order P, materials,
    a torch-owned device workspace, and the stepping calls."""

    def __init__(self, VX, EToV, N, P, rho, c, face_bc=None, periodic=None, box=None,
                 gamma=None, device=0, precision=0, n_shots=1):
        self.lib = load()
        h = C.c_void_p()
        st = self.lib.dgh_create(C.byref(h), device, precision, n_shots)
        if st != DGH_OK:
            raise DghError(f"dgh_create failed: {STATUS.get(st, st)}")
        self.h = h
        self.device = device
        self.precision = precision
        VX = np.ascontiguousarray(VX, dtype=np.float64)
        EToV = np.ascontiguousarray(EToV, dtype=np.int32)
        if box is None:
            box = np.concatenate([VX.min(axis=0), VX.max(axis=0)])
        box = np.ascontiguousarray(box, dtype=np.float64).ravel()
        per = None if periodic is None else np.ascontiguousarray(
            [1 if p else 0 for p in periodic], dtype=np.int32)
        self._call("dgh_upload_mesh", VX.shape[0], _ptr(VX), EToV.shape[0], _ptr(EToV),
                   _ptr(box), _ptr(per))
        self._call("dgh_set_order", N)
        fb = None
        if face_bc is not None:
            fb = np.ascontiguousarray([BC[b] if isinstance(b, str) else int(b) for b in face_bc],
                                      dtype=np.int32)
        g = None if gamma is None else np.ascontiguousarray(gamma, dtype=np.float64)
        self._call("dgh_set_habc", P, _ptr(g), _ptr(fb))
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        c = np.ascontiguousarray(c, dtype=np.float64)
        self._call("dgh_set_material", _ptr(rho), _ptr(c))
        cnt = np.zeros(len(COUNTS), dtype=np.int32)
        self._call("dgh_counts", _ptr(cnt))
        self.counts = dict(zip(COUNTS, (int(v) for v in cnt)))
        self.ws = None

    # ------------------------------------------------------------------
    def _call(self, name, *args):
        st = getattr(self.lib, name)(self.h, *args)
        if st != DGH_OK:
            msg = self.lib.dgh_last_error(self.h).decode()
            raise DghError(f"{name}: {STATUS.get(st, st)}: {msg}")

    def shapes(self):
        k = self.counts
        P = k["P"]
        return {
            "q3": (k["K"], 4, k["Np"]), "res3": (k["K"], 4, k["Np"]),
            "q2": (k["Ktri"], P, 3, k["Np2"]), "res2": (k["Ktri"], P, 3, k["Np2"]),
            "qb3": (k["Ktri"], k["Np2"]), "q0_3": (k["Ktri"], k["Np2"]),
            "q1": (k["Klin"], P * P, 2, k["Np1"]), "res1": (k["Klin"], P * P, 2, k["Np1"]),
            "qb2": (k["Klin"], 2, P, k["Np1"]), "q0_2": (k["Klin"], 2, P, k["Np1"]),
            "qb1": (k["Kpnt"], 3, P * P),
        }

    def node_coords(self):
        out = np.empty((self.counts["K"], self.counts["Np"], 3))
        self._call("dgh_node_coords", _ptr(out))
        return out

    def workspace_size(self):
        n = C.c_size_t()
        self._call("dgh_workspace_size", C.byref(n))
        return n.value

    def bind(self, stream=None):
        """Allocates the workspace as a torch uint8 tensor on the device and
        binds it with the given (or current) torch stream."""
        import torch
        nbytes = self.workspace_size()
        dev = torch.device("cuda", self.device)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._call("dgh_bind_workspace", C.c_void_p(base + off), C.c_size_t(nbytes),
                   C.c_void_p(self.stream.cuda_stream))
        return self

    def set_state(self, arrays=None, shot=0):
        arrays = arrays or {}
        shapes = self.shapes()
        keep = []
        ptrs = (C.c_void_p * len(ARRAYS))()
        for i, name in enumerate(ARRAYS):
            if name in arrays and arrays[name] is not None:
                a = np.ascontiguousarray(arrays[name], dtype=np.float64)
                if a.shape != shapes[name]:
                    raise ValueError(f"{name}: shape {a.shape} != {shapes[name]}")
                keep.append(a)
                ptrs[i] = a.ctypes.data
            else:
                ptrs[i] = None
        self._call("dgh_set_state", shot, C.cast(ptrs, C.c_void_p))

    def read_fields(self, names=None, shot=0):
        shapes = self.shapes()
        names = ARRAYS if names is None else names
        out = {n: np.empty(shapes[n]) for n in names}
        ptrs = (C.c_void_p * len(ARRAYS))()
        for i, name in enumerate(ARRAYS):
            ptrs[i] = out[name].ctypes.data if name in out else None
        self._call("dgh_read_fields", shot, C.cast(ptrs, C.c_void_p))
        return out

    def set_source(self, xs, f0, t0, amp=1.0, shot=0):
        x = np.ascontiguousarray(xs, dtype=np.float64)
        self._call("dgh_set_source", shot, _ptr(x), float(f0), float(t0), float(amp))

    def step(self, n_steps, dt, t_start=0.0):
        self._call("dgh_step", int(n_steps), float(dt), float(t_start))

    def tuning_count(self):
        n = C.c_int()
        self._call("dgh_tuning_count", C.byref(n))
        return n.value

    def set_tuning(self, candidate):
        self._call("dgh_set_tuning", int(candidate))

    def autotune(self, launches=20):
        """Times every launch candidate of the 3D level, keeps the fastest;
        returns (best index, milliseconds per launch of each candidate)."""
        n = self.tuning_count()
        ms = np.zeros(n)
        best = C.c_int()
        self._call("dgh_autotune", int(launches), C.byref(best), _ptr(ms))
        return best.value, ms

    def set_graph(self, enable=True):
        """Replayed stepping: each step runs as one captured HIP graph."""
        self._call("dgh_set_graph", 1 if enable else 0)

    def energy(self, shot=0):
        e = C.c_double()
        self._call("dgh_energy", shot, C.byref(e))
        return e.value

    def check(self, e_ref=0.0, rel_tol=0.0, shot=0):
        """Returns (status name, energy): DGH_OK, DGH_ENONFINITE or
        DGH_EUNSTABLE; other failures raise."""
        e = C.c_double()
        st = self.lib.dgh_check(self.h, shot, float(e_ref), float(rel_tol), C.byref(e))
        if st not in (DGH_OK, -5, -6):
            msg = self.lib.dgh_last_error(self.h).decode()
            raise DghError(f"dgh_check: {STATUS.get(st, st)}: {msg}")
        return STATUS[st], e.value

    def set_closure(self, w=None):
        """Learned closure parameters (DGH_CLOSURE_PARAMS floats), or None to
        return to the plain method."""
        if w is None:
            self._call("dgh_set_closure", None, 0)
            return
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._call("dgh_set_closure", _ptr(w), int(w.size))

    def closure_record(self, enable=True):
        self._call("dgh_closure_record", 1 if enable else 0)

    def set_closure_memory(self, tau=None):
        """Time scales of the closure's averaged inputs (4 values), or None
        for the library's default."""
        t = None if tau is None else np.ascontiguousarray(tau, dtype=np.float64)
        if t is not None and t.size != 4:
            raise ValueError("4 time scales")
        self._call("dgh_set_closure_memory", _ptr(t))

    def closure_sample(self, shot=0):
        """(X[nodes][11], Y[nodes]) from the current state (float32): sample
        rows (the closure's 10 raw inputs, then r+) and the method's r-."""
        nn = self.counts["Ktri"] * self.counts["Np2"]
        x = np.empty((nn, 11), dtype=np.float32)
        y = np.empty(nn, dtype=np.float32)
        self._call("dgh_closure_sample", shot, _ptr(x), _ptr(y))
        return x, y

    def kernel_timing(self, enable):
        self._call("dgh_kernel_timing", 1 if enable else 0)

    def kernel_time(self, level=3):
        t = C.c_double()
        n = C.c_longlong()
        self._call("dgh_kernel_time", level, C.byref(t), C.byref(n))
        return t.value, n.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.dgh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_group(solvers, n_steps, dt, t_start=0.0):
    """Steps several bound Solvers (any mesh sizes, same N) together: one 3D
    launch per stage over all of their tiles."""
    arr = (C.c_void_p * len(solvers))(*[sv.h.value for sv in solvers])
    st = load().dgh_step_group(C.cast(arr, C.c_void_p), len(solvers), int(n_steps), float(dt),
                               float(t_start))
    if st != DGH_OK:
        msg = load().dgh_last_error(solvers[0].h).decode()
        raise DghError(f"dgh_step_group: {STATUS.get(st, st)}: {msg}")


# ---- training kernels of the closure (device tensors; no context)
CLOSURE_PARAMS = 9091


def _check(st, name):
    if st != DGH_OK:
        raise DghError(f"{name}: {STATUS.get(st, st)}")


def _stream(t):
    import torch
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def mlp_work_size(batch):
    n = C.c_size_t()
    _check(load().dgh_mlp_work_size(int(batch), C.byref(n)), "dgh_mlp_work_size")
    return n.value


def mlp_forward(W, X):
    """r- for the sample rows X[n][11] (float32 CUDA tensors) -> Y[n]."""
    import torch
    Y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(load().dgh_mlp_forward(C.c_void_p(W.data_ptr()), C.c_void_p(X.data_ptr()),
                                  int(X.shape[0]), C.c_void_p(Y.data_ptr()), _stream(X)),
           "dgh_mlp_forward")
    return Y


def mlp_grad(W, X, T, G, work, with_loss=True, bf16=False):
    """Gradient of the mean squared error into G (FP32, or BF16 products on
    the matrix cores); returns the loss (or None)."""
    loss = C.c_double()
    fn = load().dgh_mlp_grad_bf16 if bf16 else load().dgh_mlp_grad
    _check(fn(C.c_void_p(W.data_ptr()), C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
              int(X.shape[0]), C.c_void_p(G.data_ptr()), C.c_void_p(work.data_ptr()),
              C.byref(loss) if with_loss else None, _stream(X)),
           "dgh_mlp_grad_bf16" if bf16 else "dgh_mlp_grad")
    return loss.value if with_loss else None


def mlp_grad_static(W, X, T, G, with_loss=True):
    """mlp_grad with the library's own fixed work array (no allocation;
    at most MLP_STATIC_BATCH rows)."""
    loss = C.c_double()
    _check(load().dgh_mlp_grad_static(C.c_void_p(W.data_ptr()), C.c_void_p(X.data_ptr()),
                                      C.c_void_p(T.data_ptr()), int(X.shape[0]),
                                      C.c_void_p(G.data_ptr()),
                                      C.byref(loss) if with_loss else None, _stream(X)),
           "dgh_mlp_grad_static")
    return loss.value if with_loss else None


MLP_STATIC_BATCH = 4096


def mlp_adam(W, G, M, V, t, lr):
    _check(load().dgh_mlp_adam(C.c_void_p(W.data_ptr()), C.c_void_p(G.data_ptr()),
                               C.c_void_p(M.data_ptr()), C.c_void_p(V.data_ptr()), int(t),
                               float(lr), _stream(W)), "dgh_mlp_adam")
