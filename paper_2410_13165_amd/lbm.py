"""Thin ctypes binding of liblbm.so (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  PyTorch supplies the device memory (through the allocator
callbacks of lbm_params) and the stream (the current torch stream at creation).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm.so")

MAX_DIM = 4
MAX_Q = 33
MAX_MODES = 16
NSCALARS = 8

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, ENONFINITE = 0, -1, -2, -3, -4, -5
MOM_PHI, MOM_SUMS, MOM_RMSE, MOM_ENTROPY, MOM_ALL = 1, 2, 4, 8, 15
BC = {"periodic": 0, "fullway": 1, "halfway": 2}
PRECISION = {"fp64": 0, "fp32": 1, "fp32_split": 2, "fp32_hilo": 3}
WALL_DATA = {"jets": 0, "tangential": 1}
FIELD = {"none": 0, "cos_sum": 1, "exp_sum": 2, "tanh_bubble": 3}
BATCH_LAUNCH = {"per_pair": 0, "resident": 1}

_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class LbmField(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("n_modes", C.c_int32),
        ("amps", C.POINTER(C.c_double)), ("kvecs", C.POINTER(C.c_double)),
        ("phases", C.POINTER(C.c_double)),
        ("Rr", C.c_double), ("W", C.c_double), ("center", C.c_double * MAX_DIM),
    ]


class LbmParams(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("dx", C.c_double), ("origin", C.c_double * MAX_DIM), ("u", C.c_double * MAX_DIM),
        ("R", C.c_double), ("g", C.c_double), ("m4", C.c_double), ("use_m4", C.c_int32),
        ("bc", (C.c_int32 * 2) * MAX_DIM), ("bc_order", C.c_int32), ("init_order", C.c_int32),
        ("precision", C.c_int32), ("field", C.POINTER(LbmField)),
        ("alloc", _ALLOC), ("free_fn", _FREE), ("alloc_ctx", C.c_void_p),
        ("stream", C.c_void_p), ("wall_data", C.c_int32), ("steps_per_pass", C.c_int32),
        ("check_every", C.c_int32),
    ]


class LbmInfo(C.Structure):
    _fields_ = [
        ("d", C.c_int32), ("q", C.c_int32), ("precision", C.c_int32),
        ("entropy_stable", C.c_int32),
        ("dims", C.c_int64 * MAX_DIM), ("nodes", C.c_int64), ("step", C.c_int64),
        ("omega", C.c_double * MAX_Q), ("m4", C.c_double), ("min_omega", C.c_double),
        ("s", C.c_double), ("dt", C.c_double), ("phi_ref", C.c_double),
        ("bytes_per_lu", C.c_int32), ("steps_per_pass", C.c_int32), ("pstride", C.c_int64),
    ]


# exported symbols and their signatures, as declared in include/lbm.h
SIGNATURES = {
    "lbm_params_default": (None, [C.POINTER(LbmParams)]),
    "lbm_create": (C.c_int, [C.c_int, C.POINTER(C.c_int64), C.c_double, C.POINTER(LbmParams),
                             C.POINTER(C.c_void_p)]),
    "lbm_set_initial": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_step_static": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_moments": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.POINTER(C.c_double)]),
    "lbm_info": (C.c_int, [C.c_void_p, C.POINTER(LbmInfo)]),
    "lbm_state_bytes": (C.c_int64, [C.c_void_p]),
    "lbm_get_state": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "lbm_equilibrium_weights": (C.c_int, [C.c_int, C.POINTER(C.c_double), C.c_double, C.c_int,
                                           C.c_double, C.POINTER(C.c_double),
                                           C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "lbm_tape_begin": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_tape_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "lbm_tape_end": (C.c_int, [C.c_void_p]),
    "lbm_profile_begin": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_profile_end": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "lbm_batch_create": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double), C.POINTER(LbmParams),
                                   C.POINTER(C.c_void_p)]),
    "lbm_batch_set_initial": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_batch_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_batch_set_launch": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "lbm_batch_tune": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int32),
                                 C.POINTER(C.c_double)]),
    "lbm_batch_instance": (C.c_void_p, [C.c_void_p, C.c_int]),
    "lbm_batch_moments": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "lbm_batch_last_error": (C.c_char_p, [C.c_void_p]),
    "lbm_batch_destroy": (C.c_int, [C.c_void_p]),
    "lbm_stability_map": (C.c_int, [C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_double,
                                    C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_bandwidth_probe": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_int64, C.c_int,
                                      C.c_int, C.c_void_p, C.POINTER(C.c_double)]),
    "lbm_probe_last_error": (C.c_char_p, []),
    "lbm_last_error": (C.c_char_p, [C.c_void_p]),
    "lbm_destroy": (C.c_int, [C.c_void_p]),
}

_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load liblbm.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_2410_13165_amd.build` "
            "(there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def equilibrium_weights(u: Sequence[float], g: float = 0.5, m4: Optional[float] = None):
    """(omega, m4, min_omega) from the library's host maths (no GPU needed)."""
    lib = load_library()
    d = len(u)
    uu = (C.c_double * max(MAX_DIM, d))(*[float(v) for v in u])
    om = (C.c_double * MAX_Q)()
    m4o = C.c_double()
    mn = C.c_double()
    rc = lib.lbm_equilibrium_weights(d, uu, float(g), 1 if m4 is not None else 0,
                                     float(m4) if m4 is not None else 0.0, om,
                                     C.byref(m4o), C.byref(mn))
    if rc != OK:
        raise LbmError(rc, lib.lbm_last_error(None).decode())
    return np.array(om[: 2 * d * d + 1]), m4o.value, mn.value


def stability_map(sigma, s, m: int = 32, g: float = 0.5, device: str = "cuda"):
    """Spectral radius of the amplification matrix over the grid xi = 2 pi j / m
    and the smallest equilibrium weight, for a batch of parameter points.

    sigma: (count, d) array of u values; s: (count,) relaxation rates (or a
    scalar).  Returns a dict of float64/int32 device tensors rho, min_omega,
    unconverged.  All work runs in the library's stability kernel.
    """
    import torch
    lib = load_library()
    sig = torch.as_tensor(sigma, dtype=torch.float64)
    if sig.dim() != 2:
        raise ValueError("sigma must be (count, d)")
    count, d = sig.shape
    ss = torch.as_tensor(s, dtype=torch.float64)
    if ss.dim() == 0:
        ss = ss.expand(count)
    if ss.shape != (count,):
        raise ValueError("s must be a scalar or have one entry per point")
    sig = sig.to(device).contiguous()
    ss = ss.to(device).contiguous()
    rho = torch.empty(count, dtype=torch.float64, device=device)
    mw = torch.empty(count, dtype=torch.float64, device=device)
    unc = torch.empty(count, dtype=torch.int32, device=device)
    stream = torch.cuda.current_stream(sig.device).cuda_stream
    rc = lib.lbm_stability_map(int(d), int(count), C.c_void_p(sig.data_ptr()),
                               C.c_void_p(ss.data_ptr()), float(g), int(m),
                               C.c_void_p(rho.data_ptr()), C.c_void_p(mw.data_ptr()),
                               C.c_void_p(unc.data_ptr()), C.c_void_p(stream))
    if rc != OK:
        raise LbmError(rc, lib.lbm_last_error(None).decode())
    return {"rho": rho, "min_omega": mw, "unconverged": unc}


def stream_ceiling(gib: float = 4.0, blocks=(1024, 4096, 16384, 65536), iters: int = 10,
                   device: str = "cuda") -> dict:
    """Best bandwidth (GB/s) of the library's float4 copy, read and write
    probes over `gib` GiB arrays and the given grid sizes."""
    import torch
    lib = load_library()
    nbytes = int(gib * (1 << 30)) // 16 * 16
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=device)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream(a.device).cuda_stream
    out = {}
    for kind, name in ((0, "copy"), (1, "read"), (2, "write")):
        best = 0.0
        for nb in blocks:
            g = C.c_double()
            rc = lib.lbm_bandwidth_probe(kind, C.c_void_p(b.data_ptr()), C.c_void_p(a.data_ptr()),
                                         nbytes, int(nb), int(iters), C.c_void_p(stream),
                                         C.byref(g))
            if rc != OK:
                raise LbmError(rc, lib.lbm_probe_last_error().decode())
            best = max(best, g.value)
        out[name] = best
    del a, b
    torch.cuda.empty_cache()
    return out


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


@dataclass
class Field:
    """Analytic solution phi*(x,t) = F(x - u t) + R t (see include/lbm.h)."""
    kind: str
    amps: Sequence[float] = ()
    kvecs: Sequence[Sequence[float]] = ()
    phases: Optional[Sequence[float]] = None
    Rr: float = 0.0
    W: float = 1.0
    center: Optional[Sequence[float]] = None

    @classmethod
    def from_dict(cls, spec: dict) -> "Field":
        return cls(kind=spec["kind"], amps=spec.get("amps", ()), kvecs=spec.get("kvecs", ()),
                   phases=spec.get("phases"), Rr=spec.get("Rr", 0.0), W=spec.get("W", 1.0),
                   center=spec.get("center"))


class Lattice:
    """One lattice of the fourth-order BGK model on the current CUDA/HIP device.

    dims = (N_1, ..., N_d); bc[a] = "periodic", "fullway" or "halfway" for both
    faces of axis a, or a pair (lower face, upper face) of them.
    """

    def __init__(self, d: int, dims: Sequence[int], tau: float = 0.5, *, dx: float,
                 u: Sequence[float], R: float = 0.0, origin: Optional[Sequence[float]] = None,
                 bc: Optional[Sequence] = None, P: int = 4, K: int = 3,
                 precision: str = "fp64", field=None, g: float = 0.5,
                 m4: Optional[float] = None, wall_data: str = "jets",
                 steps_per_pass: int = 2, check_every: int = 0, device=None):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.type != "cuda":
            raise ValueError("the lattice lives on a GPU device")
        self.d = int(d)
        self.dims = tuple(int(n) for n in dims)
        self._bufs = {}
        self._h = None
        self._closed = False

        p = LbmParams()
        self.lib.lbm_params_default(C.byref(p))
        p.dx = float(dx)
        for a in range(self.d):
            p.origin[a] = float(origin[a]) if origin is not None else 0.0
            p.u[a] = float(u[a])
            faces = bc[a] if bc is not None else "periodic"
            lo, hi = (faces, faces) if isinstance(faces, str) else faces
            p.bc[a][0], p.bc[a][1] = BC[lo], BC[hi]
        p.R = float(R)
        p.g = float(g)
        if m4 is not None:
            p.m4 = float(m4)
            p.use_m4 = 1
        p.bc_order = int(P)
        p.init_order = int(K)
        p.precision = PRECISION[precision]
        self.precision = precision
        p.wall_data = WALL_DATA[wall_data]
        p.steps_per_pass = int(steps_per_pass)
        p.check_every = int(check_every)

        self._field_keep = []
        self.n_modes = 0
        if field is not None:
            if isinstance(field, dict):
                field = Field.from_dict(field)
            f = LbmField()
            f.kind = FIELD[field.kind]
            if field.kind in ("cos_sum", "exp_sum"):
                amps = np.ascontiguousarray(field.amps, dtype=np.float64)
                kv = np.ascontiguousarray(field.kvecs, dtype=np.float64).reshape(len(amps), self.d)
                ph = np.ascontiguousarray(field.phases if field.phases is not None
                                          else np.zeros(len(amps)), dtype=np.float64)
                f.n_modes = len(amps)
                self.n_modes = len(amps)
                f.amps = amps.ctypes.data_as(C.POINTER(C.c_double))
                f.kvecs = kv.ctypes.data_as(C.POINTER(C.c_double))
                f.phases = ph.ctypes.data_as(C.POINTER(C.c_double))
                self._field_keep += [amps, kv, ph]
            f.Rr = float(field.Rr)
            f.W = float(field.W)
            if field.center is not None:
                for a in range(self.d):
                    f.center[a] = float(field.center[a])
            self._field_keep.append(f)
            p.field = C.pointer(f)

        # torch supplies the device memory
        def _alloc(nbytes, ctx):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            except RuntimeError:
                return None
            ptr = t.data_ptr()
            self._bufs[ptr] = t
            return ptr

        def _free(ptr, ctx):
            self._bufs.pop(ptr, None)

        self._alloc_cb = _ALLOC(_alloc)
        self._free_cb = _FREE(_free)
        p.alloc = self._alloc_cb
        p.free_fn = self._free_cb
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        p.stream = C.c_void_p(self.stream.cuda_stream)
        self._params = p

        dims_arr = (C.c_int64 * MAX_DIM)(*(list(self.dims) + [1] * (MAX_DIM - self.d)))
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.lbm_create(self.d, dims_arr, float(tau), C.byref(p), C.byref(h))
        if rc != OK:
            raise LbmError(rc, self.lib.lbm_last_error(None).decode())
        self._h = h

    # ------------------------------------------------------------------ ABI
    def _check(self, rc: int):
        if rc != OK:
            raise LbmError(rc, self.lib.lbm_last_error(self._h).decode())

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    @property
    def nodes(self) -> int:
        return int(np.prod(self.dims))

    def set_initial(self, phi0, grad0=None):
        torch = self._torch
        phi0 = phi0.to(device=self.device, dtype=torch.float64).contiguous()
        g = None
        if grad0 is not None:
            g = grad0.to(device=self.device, dtype=torch.float64).contiguous()
        self._check(self.lib.lbm_set_initial(self._h, C.c_void_p(phi0.data_ptr()),
                                             C.c_void_p(g.data_ptr()) if g is not None else None))
        # keep the inputs alive until the stream has consumed them
        self._init_keep = (phi0, g)
        return self

    def step(self, n: int = 1):
        self._check(self.lib.lbm_step(self._h, int(n)))
        return self

    def step_static(self, n: int = 1):
        """lbm_step_static: the same steps without any device allocation."""
        self._check(self.lib.lbm_step_static(self._h, int(n)))
        return self

    def phi(self):
        """phi(x, t_n) as a float64 tensor shaped (N_d, ..., N_1)."""
        torch = self._torch
        out = torch.empty(self.nodes, dtype=torch.float64, device=self.device)
        self._check(self.lib.lbm_moments(self._h, MOM_PHI, C.c_void_p(out.data_ptr()), None))
        return out.view(*reversed(self.dims))

    def diagnostics(self, what: int = MOM_SUMS | MOM_RMSE | MOM_ENTROPY) -> dict:
        """FP64 reductions of the current state (NaN for what `what` leaves out)."""
        vals = (C.c_double * NSCALARS)()
        self._check(self.lib.lbm_moments(self._h, int(what), None, vals))
        keys = ("sum_phi", "sum_phi2", "sum_err2", "entropy", "max_abs_phi", "nonfinite",
                "rmse", "t")
        return {k: float(v) for k, v in zip(keys, vals)}

    def info(self) -> dict:
        inf = LbmInfo()
        self._check(self.lib.lbm_info(self._h, C.byref(inf)))
        return {
            "d": inf.d, "q": inf.q, "precision": inf.precision,
            "entropy_stable": bool(inf.entropy_stable),
            "dims": tuple(inf.dims[: inf.d]), "nodes": inf.nodes, "step": inf.step,
            "omega": np.array(inf.omega[: inf.q]), "m4": inf.m4, "min_omega": inf.min_omega,
            "s": inf.s, "dt": inf.dt, "phi_ref": inf.phi_ref, "bytes_per_lu": inf.bytes_per_lu,
            "pstride": inf.pstride, "steps_per_pass": inf.steps_per_pass,
        }

    def tape_begin(self, every: int):
        self._check(self.lib.lbm_tape_begin(self._h, int(every)))
        return self

    def tape_end(self):
        self._check(self.lib.lbm_tape_end(self._h))
        return self

    def tape_gradient(self, dl_dphi, want_phi0: bool = True, want_grad0: bool = False,
                      want_tau: bool = True, want_wall: bool = False) -> dict:
        """Adjoint gradients of L given dL/dphi^N (shape (N_d, ..., N_1)).

        want_wall: dL/da_j and dL/dtheta_j of the analytic field as it enters
        the Dirichlet data ("wall_amps", "wall_phases")."""
        torch = self._torch
        seed = dl_dphi.to(device=self.device, dtype=torch.float64).contiguous()
        gphi = torch.empty(self.nodes, dtype=torch.float64, device=self.device) if want_phi0 else None
        ggrad = (torch.empty(self.d * self.nodes, dtype=torch.float64, device=self.device)
                 if want_grad0 else None)
        tau = C.c_double()
        wall = (C.c_double * (2 * MAX_MODES))()
        self._check(self.lib.lbm_tape_gradient(
            self._h, C.c_void_p(seed.data_ptr()),
            C.c_void_p(gphi.data_ptr()) if gphi is not None else None,
            C.c_void_p(ggrad.data_ptr()) if ggrad is not None else None,
            C.byref(tau) if want_tau else None,
            wall if want_wall else None))
        out = {}
        if gphi is not None:
            out["phi0"] = gphi.view(*reversed(self.dims))
        if ggrad is not None:
            out["grad0"] = ggrad.view(self.d, *reversed(self.dims))
        if want_tau:
            out["tau"] = tau.value
        if want_wall:
            m = self.n_modes
            out["wall_amps"] = np.array(wall[:m])
            out["wall_phases"] = np.array(wall[m:2 * m])
        return out

    def profile_begin(self, max_launches: int):
        self._check(self.lib.lbm_profile_begin(self._h, int(max_launches)))
        return self

    def profile_end(self) -> dict:
        b, w, n, nl = C.c_double(), C.c_double(), C.c_int64(), C.c_int64()
        self._check(self.lib.lbm_profile_end(self._h, C.byref(b), C.byref(w), C.byref(n),
                                             C.byref(nl)))
        return {"bulk_ms": b.value, "wall_ms": w.value, "steps": n.value, "launches": nl.value}

    def state_bytes(self) -> int:
        return int(self.lib.lbm_state_bytes(self._h))

    def get_state(self):
        torch = self._torch
        buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        self._check(self.lib.lbm_get_state(self._h, C.c_void_p(buf.data_ptr())))
        return buf

    def set_state(self, buf, step: int):
        self._check(self.lib.lbm_set_state(self._h, C.c_void_p(buf.data_ptr()), int(step)))
        self._state_keep = buf
        return self

    def close(self):
        if self._h is not None and not self._closed:
            self._closed = True
            self.lib.lbm_destroy(self._h)
            self._h = None
            self._bufs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _BatchMember(Lattice):
    """Read-only view of one instance of a Batch (moments, info, state)."""

    def __init__(self, batch, handle, d, dims, precision, R):
        self._torch = batch._torch
        self.lib = batch.lib
        self.device = batch.device
        self.d = d
        self.dims = tuple(dims)
        self.precision = precision
        self._h = C.c_void_p(handle)
        self._closed = True  # owned by the batch
        self._bufs = {}
        p = LbmParams()
        p.R = R
        self._params = p

    def close(self):
        pass


class Batch:
    """Independent periodic lattices of one d and precision advanced together.

    specs: list of dicts with keys dims, tau, dx, u and optional R, m4, g, K and
    steps_per_pass (2 by default: d = 2 batches advance two steps per pass).
    """

    def __init__(self, d: int, specs, precision: str = "fp32", device=None):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.device = torch.device(device if device is not None else "cuda")
        self.d = int(d)
        self.count = len(specs)
        self._bufs = {}
        self._b = None

        def _alloc(nbytes, ctx):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            except RuntimeError:
                return None
            self._bufs[t.data_ptr()] = t
            return t.data_ptr()

        def _free(ptr, ctx):
            self._bufs.pop(ptr, None)

        self._alloc_cb = _ALLOC(_alloc)
        self._free_cb = _FREE(_free)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        params = (LbmParams * self.count)()
        dims = (C.c_int64 * (self.count * self.d))()
        taus = (C.c_double * self.count)()
        self.specs = [dict(sp) for sp in specs]
        for i, sp in enumerate(self.specs):
            p = params[i]
            self.lib.lbm_params_default(C.byref(p))
            p.dx = float(sp["dx"])
            for a in range(self.d):
                p.u[a] = float(sp["u"][a])
                dims[i * self.d + a] = int(sp["dims"][a])
            p.R = float(sp.get("R", 0.0))
            p.g = float(sp.get("g", 0.5))
            if sp.get("m4") is not None:
                p.m4 = float(sp["m4"])
                p.use_m4 = 1
            p.init_order = int(sp.get("K", 1))
            p.steps_per_pass = int(sp.get("steps_per_pass", 2))
            p.precision = PRECISION[precision]
            p.alloc = self._alloc_cb
            p.free_fn = self._free_cb
            p.stream = C.c_void_p(self.stream.cuda_stream)
            taus[i] = float(sp["tau"])
        self.precision = precision
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.lbm_batch_create(self.count, self.d, dims, taus, params, C.byref(h))
        if rc != OK:
            raise LbmError(rc, self.lib.lbm_batch_last_error(None).decode())
        self._b = h
        self._params = params
        self.nodes = [int(np.prod(sp["dims"])) for sp in self.specs]

    def _check(self, rc):
        if rc != OK:
            raise LbmError(rc, self.lib.lbm_batch_last_error(self._b).decode())

    def set_initial(self, phi0_concat, grad_concat=None):
        torch = self._torch
        phi = phi0_concat.to(device=self.device, dtype=torch.float64).contiguous()
        g = None if grad_concat is None else grad_concat.to(device=self.device,
                                                            dtype=torch.float64).contiguous()
        self._check(self.lib.lbm_batch_set_initial(
            self._b, C.c_void_p(phi.data_ptr()), C.c_void_p(g.data_ptr()) if g is not None else None))
        self._keep = (phi, g)
        return self

    def step(self, n: int):
        self._check(self.lib.lbm_batch_step(self._b, int(n)))
        return self

    def tune(self, trial_steps: int = 10) -> dict:
        """lbm_batch_tune: time every launch form and tile shape, keep the fastest."""
        cfg = (C.c_int32 * 5)()
        ms = C.c_double()
        self._check(self.lib.lbm_batch_tune(self._b, int(trial_steps), cfg, C.byref(ms)))
        form = {0: "per_pair", 1: "resident"}.get(cfg[0])
        return {"form": form, "ychunk": cfg[1], "tx": cfg[2], "ty": cfg[3],
                "cached": bool(cfg[4]), "ms_per_step": ms.value}

    def set_launch(self, form: str = "per_pair", ychunk: int = 0):
        """lbm_batch_set_launch: "per_pair" launches or one "resident" launch per call."""
        self._check(self.lib.lbm_batch_set_launch(self._b, BATCH_LAUNCH[form], int(ychunk)))
        return self

    def moments(self) -> np.ndarray:
        out = (C.c_double * (NSCALARS * self.count))()
        self._check(self.lib.lbm_batch_moments(self._b, out))
        return np.array(out[:]).reshape(self.count, NSCALARS)

    def instance(self, i: int) -> Lattice:
        h = self.lib.lbm_batch_instance(self._b, int(i))
        if not h:
            raise IndexError(i)
        sp = self.specs[i]
        return _BatchMember(self, h, self.d, sp["dims"], self.precision, float(sp.get("R", 0.0)))

    def close(self):
        if self._b is not None:
            self.lib.lbm_batch_destroy(self._b)
            self._b = None
            self._bufs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
