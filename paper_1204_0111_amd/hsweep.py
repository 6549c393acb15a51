"""Python binding of libhsweep (the C ABI in include/hsweep.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies device memory and the stream.  Importing works without a
GPU; creating a Solver needs the built library and a device, and raises if
either is missing (there is no fallback).
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsweep.so")

HSW_C128, HSW_C64, HSW_C64_BF16GEMM = 0, 1, 2
PRECISIONS = {"c128": HSW_C128, "c64": HSW_C64, "c64_bf16": HSW_C64_BF16GEMM}
STATUS = {0: "HSW_OK", 1: "HSW_E_INVAL", 2: "HSW_E_NOMEM", 3: "HSW_E_STATE",
          4: "HSW_E_BREAKDOWN", 5: "HSW_E_NOCONV", 6: "HSW_E_DEVICE"}

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class HswProblem(ctypes.Structure):
    _fields_ = [("n", c_int32 * 3), ("h", c_double), ("omega", c_double), ("alpha", c_double),
                ("gamma", c_int32), ("pml_amp", c_double), ("panel_depth", c_int32),
                ("leaf", c_int32)]


class HswSolveOpts(ctypes.Structure):
    _fields_ = [("restart_k", c_int32), ("maxit", c_int32), ("rtol", c_double)]


class HswSolveInfo(ctypes.Structure):
    _fields_ = [("iters_max", c_int32), ("iters", ctypes.POINTER(c_int32)),
                ("relres", ctypes.POINTER(c_double)), ("t_setup", c_double),
                ("t_solve", c_double), ("bad_problem", c_int32), ("bad_panel", c_int32),
                ("bad_front", c_int32), ("bad_pivot", c_int32)]


class HswError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


_lib = None


def load_library():
    """Load libhsweep.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhsweep.so is not built: run `python -m paper_1204_0111_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "hsw_create": (c_int32, [P(HswProblem), c_int32, c_int32, c_void_p, P(c_void_p)]),
        "hsw_assemble": (c_int32, [c_void_p, P(c_void_p)]),
        "hsw_setup": (c_int32, [c_void_p]),
        "hsw_apply": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_int64]),
        "hsw_apply_noalloc": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_int64]),
        "hsw_panel_solve": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_int32,
                                      c_int64]),
        "hsw_matvec": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_int64]),
        "hsw_solve": (c_int32, [c_void_p, P(c_void_p), P(c_void_p), P(c_int32), P(HswSolveOpts),
                                P(HswSolveInfo)]),
        "hsw_query": (c_int32, [c_void_p, c_int32, ctypes.c_char_p, P(c_int64)]),
        "hsw_get_perm": (c_int32, [c_void_p, c_int32, c_int32, P(c_int32)]),
        "hsw_get_front_info": (c_int32, [c_void_p, c_int32, c_int32, c_int32, P(c_int32),
                                         P(c_int32)]),
        "hsw_get_front": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                    c_void_p, P(c_int32), P(c_int32)]),
        "hsw_get_front_inverse": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p]),
        "hsw_kernel_timing": (c_int32, [c_void_p, ctypes.c_char_p, c_int32, P(c_int64),
                                        P(c_double), P(c_double), P(c_double)]),
        "hsw_set_option": (c_int32, [c_void_p, ctypes.c_char_p, c_int64]),
        "hsw_last_error": (ctypes.c_char_p, [c_void_p]),
        "hsw_destroy": (None, [c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _problem_struct(p):
    s = HswProblem()
    for j in range(3):
        s.n[j] = int(p["n"][j])
    s.h = float(p["h"])
    s.omega = float(p["omega"])
    s.alpha = float(p.get("alpha", 0.0))
    s.gamma = int(p["gamma"])
    s.pml_amp = float(p.get("C", p.get("pml_amp", 0.0)))
    s.panel_depth = int(p["d"] if "d" in p else p["panel_depth"])
    s.leaf = int(p.get("leaf", 4))
    return s


class Solver:
    """One context: plan + factors of one or more problems on the current device.

    problems: dicts with n (3 ints), h, omega, alpha, gamma, C (PML amplitude),
    d (panel depth), leaf.  precision: "c128", "c64" or "c64_bf16".
    """

    def __init__(self, problems, precision="c64", stream=None):
        import torch
        self._torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("hsweep needs a HIP device")
        self.lib = load_library()
        if isinstance(problems, dict):
            problems = [problems]
        self.problems = [dict(p) for p in problems]
        arr = (HswProblem * len(problems))(*[_problem_struct(p) for p in problems])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        ctx = c_void_p()
        st = self.lib.hsw_create(arr, len(problems), PRECISIONS[precision],
                                 c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if st != 0:
            raise HswError(st, self.lib.hsw_last_error(None).decode())
        self.ctx = ctx
        self.precision = precision
        self._keep = []

    # -- helpers ------------------------------------------------------------
    def _check(self, st):
        if st != 0:
            raise HswError(st, self.lib.hsw_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.hsw_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, prob, key, val=0):
        v = c_int64(val)
        self._check(self.lib.hsw_query(self.ctx, prob, key.encode(), ctypes.byref(v)))
        return v.value

    def N_pad(self, prob=0):
        return self.query(prob, "N_pad")

    def _cvec(self, x, n, name):
        t = self._torch
        x = t.as_tensor(x)
        if x.dim() == 1:
            x = x.unsqueeze(0)
        if x.dtype != t.complex128 or x.device.type != "cuda" or not x.is_contiguous() \
                or x.shape[1] != n:
            raise ValueError("%s must be a contiguous complex128 CUDA tensor of shape (nrhs, %d)"
                             % (name, n))
        return x

    # -- the C calls ----------------------------------------------------------
    def assemble(self, velocities):
        t = self._torch
        if not isinstance(velocities, (list, tuple)):
            velocities = [velocities]
        dev = []
        for c in velocities:
            ct = t.as_tensor(np.ascontiguousarray(c) if isinstance(c, np.ndarray) else c,
                             dtype=t.float64).to("cuda").contiguous()
            dev.append(ct)
        ptrs = (c_void_p * len(dev))(*[c_void_p(c.data_ptr()) for c in dev])
        self._check(self.lib.hsw_assemble(self.ctx, ptrs))
        self.stream.synchronize()

    def setup(self):
        self._check(self.lib.hsw_setup(self.ctx))

    def apply(self, prob, r, out=None):
        n = self.N_pad(prob)
        r = self._cvec(r, n, "r")
        z = self._torch.empty_like(r) if out is None else out
        self._check(self.lib.hsw_apply(self.ctx, prob, c_void_p(r.data_ptr()),
                                       c_void_p(z.data_ptr()), r.shape[0], n))
        return z

    def apply_noalloc(self, prob, r, out):
        """hsw_apply_noalloc: the sweep with the library's static device
        scratch as workspace (no allocation; at most 15 right-hand sides)."""
        n = self.N_pad(prob)
        r = self._cvec(r, n, "r")
        out = self._cvec(out, n, "out")
        self._check(self.lib.hsw_apply_noalloc(self.ctx, prob, c_void_p(r.data_ptr()),
                                               c_void_p(out.data_ptr()), r.shape[0], n))
        return out

    def matvec(self, prob, x):
        n = self.N_pad(prob)
        x = self._cvec(x, n, "x")
        y = self._torch.empty_like(x)
        self._check(self.lib.hsw_matvec(self.ctx, prob, c_void_p(x.data_ptr()),
                                        c_void_p(y.data_ptr()), x.shape[0], n))
        return y

    def panel_solve(self, prob, panel, v):
        lo = self.query(prob, "panel_lo", panel)
        hi = self.query(prob, "panel_hi", panel)
        n = (hi - lo) * self.query(prob, "N1") * self.query(prob, "N2")
        v = self._cvec(v, n, "v")
        y = self._torch.empty_like(v)
        self._check(self.lib.hsw_panel_solve(self.ctx, prob, panel, c_void_p(v.data_ptr()),
                                             c_void_p(y.data_ptr()), v.shape[0], n))
        return y

    def solve(self, bs, rtol=1e-5, restart=20, maxit=1000):
        """GMRES for every problem; bs[k]: (nrhs_k, N_pad) complex128 CUDA tensor."""
        t = self._torch
        if not isinstance(bs, (list, tuple)):
            bs = [bs]
        bs = [self._cvec(b, self.N_pad(k), "b") for k, b in enumerate(bs)]
        xs = [t.empty_like(b) for b in bs]
        nr = (c_int32 * len(bs))(*[b.shape[0] for b in bs])
        tot = sum(b.shape[0] for b in bs)
        iters = (c_int32 * tot)()
        relres = (c_double * tot)()
        info = HswSolveInfo()
        info.iters = ctypes.cast(iters, ctypes.POINTER(c_int32))
        info.relres = ctypes.cast(relres, ctypes.POINTER(c_double))
        opts = HswSolveOpts(restart, maxit, rtol)
        bp = (c_void_p * len(bs))(*[c_void_p(b.data_ptr()) for b in bs])
        xp = (c_void_p * len(bs))(*[c_void_p(x.data_ptr()) for x in xs])
        st = self.lib.hsw_solve(self.ctx, bp, xp, nr, ctypes.byref(opts), ctypes.byref(info))
        if st not in (0, 5):
            self._check(st)
        out = dict(status=STATUS[st], iters=list(iters), relres=list(relres),
                   iters_max=info.iters_max, t_setup=info.t_setup, t_solve=info.t_solve)
        return xs, out

    def perm(self, prob, panel):
        naux = self.query(prob, "panel_naux", panel)
        out = np.empty(naux, dtype=np.int32)
        self._check(self.lib.hsw_get_perm(self.ctx, prob, panel,
                                          out.ctypes.data_as(ctypes.POINTER(c_int32))))
        return out

    def front_info(self, prob, panel, front):
        info = np.empty(5, dtype=np.int32)
        self._check(self.lib.hsw_get_front_info(self.ctx, prob, panel, front,
                                                info.ctypes.data_as(ctypes.POINTER(c_int32)),
                                                None))
        u = np.empty(max(int(info[2]), 1), dtype=np.int32)
        self._check(self.lib.hsw_get_front_info(self.ctx, prob, panel, front,
                                                info.ctypes.data_as(ctypes.POINTER(c_int32)),
                                                u.ctypes.data_as(ctypes.POINTER(c_int32))))
        return dict(start=int(info[0]), s=int(info[1]), u=int(info[2]), parent=int(info[3]),
                    depth=int(info[4]), urows=u[:int(info[2])].copy())

    def front(self, prob, panel, front):
        fi = self.front_info(prob, panel, front)
        s, u = fi["s"], fi["u"]
        D = np.empty(s, dtype=np.complex128)
        L = np.empty((s, s), dtype=np.complex128, order="F")
        F = np.empty((max(u, 1), s), dtype=np.complex128, order="F")
        self._check(self.lib.hsw_get_front(self.ctx, prob, panel, front, c_void_p(D.ctypes.data),
                                           c_void_p(L.ctypes.data), c_void_p(F.ctypes.data),
                                           None, None))
        return D, L, F[:u]

    def set_option(self, key, value):
        """Option of the context: "graph", "autotune", "update_order", "block_gmres",
        "solve_lanes", "keep_factors", "inverse_by_depth", "full_inverse",
        "triangular_solves", "bf16_mfma", "mm_min_rhs", "mm_fwd_form", "mm_bwd_form" or
        "gmres_device_test" (see hsw_set_option)."""
        self._check(self.lib.hsw_set_option(self.ctx, key.encode(), int(value)))

    def kernel_timing(self, kernel, enable):
        """Start (enable=True) or stop timing a kernel class; stopping returns the totals."""
        n = c_int64()
        sec, byt, fl = c_double(), c_double(), c_double()
        self._check(self.lib.hsw_kernel_timing(self.ctx, kernel.encode(), int(bool(enable)),
                                               ctypes.byref(n), ctypes.byref(sec),
                                               ctypes.byref(byt), ctypes.byref(fl)))
        return dict(launches=n.value, seconds=sec.value, bytes=byt.value, flops=fl.value)

    def front_inverse(self, prob, panel, front):
        fi = self.front_info(prob, panel, front)
        G = np.empty((fi["s"] + fi["u"], fi["s"]), dtype=np.complex128, order="F")
        self._check(self.lib.hsw_get_front_inverse(self.ctx, prob, panel, front,
                                                   c_void_p(G.ctypes.data)))
        return G
