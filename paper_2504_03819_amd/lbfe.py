"""ctypes binding of the lbfe C ABI (include/lbfe.h).

Argument marshalling only: every step of the method runs in the HIP library
``_lib/liblbfe.so``.  torch supplies device memory (the workspace and the
field / state buffers) and the HIP stream; nothing here computes physics.
"""
import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

LIB_PATH = os.environ.get("LBFE_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "liblbfe.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_DIVERGED, E_STATE = 0, -1, -2, -3, -4, -5
FP64, FP32, FP16_DEV, FP16_DEV_F0FP32 = 0, 1, 2, 3
WET_NEUTRAL, WET_PHI, WET_DELTA = 0, 1, 2
AUTO, PATH_TWO_PASS, PATH_FUSED, PATH_STATE = 0, 1, 2, 3
ORDER_ROUND_ROBIN, ORDER_XCD = 1, 2
FIELD_RHO, FIELD_U, FIELD_MU, FIELD_F, FIELD_Q, FIELD_PM = 0, 1, 2, 3, 4, 5
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16dev": FP16_DEV, "fp16dev_f0fp32": FP16_DEV_F0FP32}
_CODES = {E_INVAL: "LBFE_E_INVAL", E_NOMEM: "LBFE_E_NOMEM", E_DEVICE: "LBFE_E_DEVICE",
          E_DIVERGED: "LBFE_E_DIVERGED", E_STATE: "LBFE_E_STATE"}


class LBFEError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    """Mirror of struct lbfe_params."""
    _fields_ = [
        ("nx", c_int64), ("ny", c_int64), ("nz", c_int64),
        ("walls_z", c_int32), ("precision", c_int32),
        ("a", c_double), ("b", c_double), ("R", c_double), ("T", c_double),
        ("kappa", c_double), ("nu", c_double), ("omega", c_double * 11),
        ("corr4", c_int32), ("wet_mode", c_int32), ("wet_value", c_double),
        ("rho_l", c_double), ("rho_v", c_double),
        ("check_every", c_int32), ("adjoint", c_int32),
        ("wall_u", c_double * 4),
        ("solid_mask", c_int32),
        ("step_path", c_int32), ("tile_order", c_int32), ("chain_chunk", c_int32),
    ]


_lib = None


def lib():
    """Load liblbfe.so (built in-tree by __graft_entry__.build()); raises if
    it is missing: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, V = POINTER(Params), c_void_p
    sig = {
        "lbfe_params_default": (c_int, [P]),
        "lbfe_coexistence": (c_int, [c_double, c_double, c_double, c_double, POINTER(c_double), POINTER(c_double)]),
        "lbfe_create": (c_int, [P, V, POINTER(V)]),
        "lbfe_workspace_bytes": (c_int, [P, POINTER(c_size_t)]),
        "lbfe_bind_workspace": (c_int, [V, V, c_size_t]),
        "lbfe_get_params": (c_int, [V, P]),
        "lbfe_set_solid": (c_int, [V, V]),
        "lbfe_init_density": (c_int, [V, V, V]),
        "lbfe_step": (c_int, [V, c_int64]),
        "lbfe_step_count": (c_int, [V, POINTER(c_int64)]),
        "lbfe_step_timed": (c_int, [V, c_int64, POINTER(c_double)]),
        "lbfe_fields": (c_int, [V, V, V, V, V]),
        "lbfe_field": (c_int, [V, c_int, V]),
        "lbfe_state_bytes": (c_int, [V, POINTER(c_size_t)]),
        "lbfe_get_state": (c_int, [V, V]),
        "lbfe_set_state": (c_int, [V, V, c_int64]),
        "lbfe_get_populations": (c_int, [V, V]),
        "lbfe_set_populations": (c_int, [V, V]),
        "lbfe_reduce": (c_int, [V, POINTER(c_double)]),
        "lbfe_reduce_into": (c_int, [V, V]),
        "lbfe_adjoint_seed": (c_int, [V, V]),
        "lbfe_adjoint_step": (c_int, [V, V]),
        "lbfe_adjoint_seed_populations": (c_int, [V, V]),
        "lbfe_adjoint_get": (c_int, [V, V]),
        "lbfe_adjoint_init_density": (c_int, [V, V, V, V]),
        "lbfe_adjoint_grads": (c_int, [V, POINTER(c_double)]),
        "lbfe_aux_bytes": (c_int, [V, POINTER(c_size_t)]),
        "lbfe_step_aux": (c_int, [V, V]),
        "lbfe_adjoint_step_aux": (c_int, [V, V, V]),
        "lbfe_last_error": (ctypes.c_char_p, [V]),
        "lbfe_destroy": (c_int, [V]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def default_params(**kw):
    p = Params()
    rc = lib().lbfe_params_default(byref(p))
    assert rc == OK
    for k, v in kw.items():
        if k in ("omega", "wall_u"):
            arr = getattr(p, k)
            for i, w in enumerate(v):
                arr[i] = float(w)
        elif k == "precision" and isinstance(v, str):
            p.precision = PRECISIONS[v]
        else:
            setattr(p, k, v)
    return p


def coexistence(a, b, R, T):
    rl, rv = c_double(), c_double()
    rc = lib().lbfe_coexistence(a, b, R, T, byref(rl), byref(rv))
    if rc != OK:
        raise LBFEError(rc, "no coexistence pair at this temperature")
    return rl.value, rv.value


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(None)


class Simulation:
    """One lbfe context with a torch-owned workspace on a CUDA/HIP device.

    All calls are enqueued on the torch stream that is current at
    construction; tensors passed in must live on the same device."""

    def __init__(self, params=None, device="cuda", solid=None, **kw):
        """solid: optional (nz, ny, nx) mask (nonzero = solid voxel), which
        sets params.solid_mask and is handed to lbfe_set_solid."""
        import torch
        self._torch = torch
        if solid is not None:
            kw["solid_mask"] = 1
        self.params = params if params is not None else default_params(**kw)
        if params is not None and kw:
            raise ValueError("give params or keyword overrides, not both")
        self.device = torch.device(device)
        L = lib()
        self._ctx = c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device)
            self.stream = stream
            rc = L.lbfe_create(byref(self.params), c_void_p(stream.cuda_stream), byref(self._ctx))
            if rc != OK:
                raise LBFEError(rc, "lbfe_create failed (parameters or device)")
            nb = c_size_t()
            self._check(L.lbfe_workspace_bytes(byref(self.params), byref(nb)))
            self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) & ~255
            self._check(L.lbfe_bind_workspace(self._ctx, c_void_p(aligned), c_size_t(nb.value)))
        q = Params()
        self._check(L.lbfe_get_params(self._ctx, byref(q)))
        self.params = q
        self.shape = (int(q.nz), int(q.ny), int(q.nx))
        if solid is not None:
            self.set_solid(solid)

    def set_solid(self, mask):
        """Give the solid voxel mask (nonzero = solid); discards the state."""
        m = self._dev(self._torch.as_tensor(mask) != 0, dtype=self._torch.uint8)
        self._check(lib().lbfe_set_solid(self._ctx, _ptr(m)))
        self.solid = m

    # -------------------------------------------------------------- utils --
    def _check(self, rc):
        if rc != OK:
            msg = lib().lbfe_last_error(self._ctx).decode()
            raise LBFEError(rc, msg)

    def _dev(self, t, comps=1, dtype=None):
        torch = self._torch
        dtype = dtype or torch.float64
        shape = ((comps,) if comps > 1 else ()) + self.shape
        if t is None:
            return None
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(t)
        t = t.to(device=self.device, dtype=dtype).contiguous()
        if tuple(t.shape) != shape:
            t = t.reshape(shape)
        return t

    def _empty(self, comps=1):
        shape = ((comps,) if comps > 1 else ()) + self.shape
        return self._torch.empty(shape, dtype=self._torch.float64, device=self.device)

    @property
    def rho_l(self):
        return self.params.rho_l

    @property
    def rho_v(self):
        return self.params.rho_v

    # ------------------------------------------------------------ forward --
    def init_density(self, rho0, u0=None):
        self._rho0 = self._dev(rho0)
        self._u0 = self._dev(u0, 3)
        self._check(lib().lbfe_init_density(self._ctx, _ptr(self._rho0), _ptr(self._u0)))

    def step(self, n=1):
        self._check(lib().lbfe_step(self._ctx, c_int64(int(n))))

    KERNELS = ("moments", "chain", "collide_stream", "wall_rho")

    def step_timed(self, n):
        """Run n steps with HIP events around each kernel; returns the summed
        milliseconds per kernel class."""
        out = (c_double * 4)()
        self._check(lib().lbfe_step_timed(self._ctx, c_int64(int(n)), out))
        return dict(zip(self.KERNELS, list(out)))

    @property
    def step_count(self):
        s = c_int64()
        self._check(lib().lbfe_step_count(self._ctx, byref(s)))
        return s.value

    def field(self, which):
        comps = 3 if which in (FIELD_U, FIELD_F, FIELD_Q) else 1
        out = self._empty(comps)
        self._check(lib().lbfe_field(self._ctx, int(which), _ptr(out)))
        return out

    def fields(self):
        rho, u, mu, F = self._empty(), self._empty(3), self._empty(), self._empty(3)
        self._check(lib().lbfe_fields(self._ctx, _ptr(rho), _ptr(u), _ptr(mu), _ptr(F)))
        return {"rho": rho, "u": u, "mu": mu, "F": F}

    def populations(self):
        out = self._torch.empty((27,) + self.shape, dtype=self._torch.float64, device=self.device)
        self._check(lib().lbfe_get_populations(self._ctx, _ptr(out)))
        return out

    def set_populations(self, f):
        f = self._dev(f, 27)
        self._keep = f
        self._check(lib().lbfe_set_populations(self._ctx, _ptr(f)))

    def state_bytes(self):
        n = c_size_t()
        self._check(lib().lbfe_state_bytes(self._ctx, byref(n)))
        return n.value

    def get_state(self, out=None):
        if out is None:
            out = self._torch.empty(self.state_bytes(), dtype=self._torch.uint8, device=self.device)
        self._check(lib().lbfe_get_state(self._ctx, _ptr(out)))
        return out

    def set_state(self, src, step=0):
        self._check(lib().lbfe_set_state(self._ctx, _ptr(src), c_int64(int(step))))

    def reduce(self):
        out = (c_double * 8)()
        self._check(lib().lbfe_reduce(self._ctx, out))
        return list(out)

    def reduce_into(self, out):
        """lbfe_reduce_into: the 8 reductions into the device tensor `out`
        (float64, 8 elements), asynchronously; no allocation."""
        torch = self._torch
        if out.dtype != torch.float64 or out.numel() < 8 or not out.is_contiguous() or out.device != self.device:
            raise ValueError("out must be a contiguous float64 device tensor of >= 8 elements on the context's device")
        self._check(lib().lbfe_reduce_into(self._ctx, _ptr(out)))
        return out

    # ------------------------------------------------------------ adjoint --
    def adjoint_seed(self, dL_drho):
        g = self._dev(dL_drho)
        self._keep_seed = g
        self._check(lib().lbfe_adjoint_seed(self._ctx, _ptr(g)))

    def adjoint_seed_populations(self, dL_df):
        g = self._dev(dL_df, 27)
        self._keep_seed = g
        self._check(lib().lbfe_adjoint_seed_populations(self._ctx, _ptr(g)))

    def adjoint_state(self):
        out = self._torch.empty((27,) + self.shape, dtype=self._torch.float64, device=self.device)
        self._check(lib().lbfe_adjoint_get(self._ctx, _ptr(out)))
        return out

    def adjoint_step(self, state_t=None):
        """One adjoint step with f(t) = state_t, or the current state if None."""
        self._check(lib().lbfe_adjoint_step(self._ctx, _ptr(state_t)))

    # ------------------------------------- forward fields kept for the adjoint --
    def aux_record(self):
        """A device buffer (uint8, 256-byte aligned view) for one record of
        the forward auxiliary fields (lbfe_aux_bytes)."""
        n = c_size_t()
        self._check(lib().lbfe_aux_bytes(self._ctx, byref(n)))
        raw = self._torch.empty(n.value + 256, dtype=self._torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        return raw[off:off + n.value]

    def step_aux(self, record):
        """One step; the fields of the state before it go into `record`."""
        self._check(lib().lbfe_step_aux(self._ctx, _ptr(record)))

    def adjoint_step_aux(self, state_t, record):
        """adjoint_step with the record that step_aux left for state_t."""
        self._check(lib().lbfe_adjoint_step_aux(self._ctx, _ptr(state_t), _ptr(record)))

    def adjoint_init_density(self, rho0=None, u0=None):
        """dL/drho0 for the initial state made by init_density (the rho0 and
        u0 given there are reused unless passed again)."""
        if rho0 is None:
            rho0, u0 = self._rho0, self._u0
        else:
            rho0, u0 = self._dev(rho0), self._dev(u0, 3)
        out = self._empty()
        self._check(lib().lbfe_adjoint_init_density(self._ctx, _ptr(rho0), _ptr(u0), _ptr(out)))
        return out

    def adjoint_grads(self):
        out = (c_double * 4)()
        self._check(lib().lbfe_adjoint_grads(self._ctx, out))
        return {"kappa": out[0], "wet_value": out[1], "nu": out[2]}

    # ------------------------------------------------------------ cleanup --
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            lib().lbfe_destroy(self._ctx)
            self._ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
