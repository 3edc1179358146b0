"""ctypes binding of libsdpm (include/sdpm.h).  Argument marshalling only:
every step of the particle-mesh path runs in the library's HIP kernels.
PyTorch supplies device memory and the stream.

The library must have been built (``python -m paper_1709_04703_amd.build``);
loading fails loudly otherwise - there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdpm.so")

SDPM_OK, SDPM_EINVAL, SDPM_ENOMEM, SDPM_EHIP = 0, -1, -2, -3
SDPM_ENOCONV, SDPM_EDOMAIN, SDPM_EOVERFLOW, SDPM_ESTATE, SDPM_EFULL = -4, -5, -6, -7, -8
SDPM_MIXED, SDPM_PLAIN_FP64 = 0, 1
SDPM_WS_PREV, SDPM_WS_LEARNED, SDPM_WS_LEARNED_GATED, SDPM_WS_EXTRAP = 0, 1, 2, 4
SDPM_SOLVER_IMPLICIT, SDPM_SOLVER_ADE, SDPM_SOLVER_FFT = 0, 1, 2
SDPM_ASSIGN_CIC, SDPM_ASSIGN_TSC = 0, 1
SDPM_PK_SHOT, SDPM_PK_JING = 1, 2

ERROR_NAMES = {
    SDPM_EINVAL: "EINVAL", SDPM_ENOMEM: "ENOMEM", SDPM_EHIP: "EHIP",
    SDPM_ENOCONV: "ENOCONV", SDPM_EDOMAIN: "EDOMAIN", SDPM_EOVERFLOW: "EOVERFLOW",
    SDPM_ESTATE: "ESTATE", SDPM_EFULL: "EFULL",
}

# every symbol include/sdpm.h declares
EXPORTS = [
    "sdpm_step_scalars", "sdpm_lightcone_radius", "sdpm_domain_box", "sdpm_config_default",
    "sdpm_workspace_bytes", "sdpm_create", "sdpm_bind", "sdpm_init_potential", "sdpm_step",
    "sdpm_shrink", "sdpm_shrink_radius", "sdpm_get_state", "sdpm_deposit", "sdpm_solve",
    "sdpm_interp_force", "sdpm_sort", "sdpm_set_warmstart_weights", "sdpm_conv3d",
    "sdpm_conv3d_wgrad", "sdpm_net_scratch_bytes", "sdpm_net_prep", "sdpm_net_forward",
    "sdpm_net_forward_noalloc", "sdpm_net_train_step", "sdpm_record", "sdpm_record_info", "sdpm_profile", "sdpm_profile_read",
    "sdpm_destroy", "sdpm_last_error", "sdpm_set_lightcone", "sdpm_lightcone_count",
    "sdpm_ade_sweep", "sdpm_pk_workspace_bytes", "sdpm_power_spectrum", "sdpm_profile_kernels",
    "sdpm_rb_sweeps",
]
NET_PARAMS = 5 * (27 * 16 * 16 + 16)
CONV_RELU, CONV_OUT_FP32_CH0, CONV_BACKWARD_DATA, CONV_MASK = 1, 2, 4, 8


class Config(ctypes.Structure):
    _fields_ = [
        ("ng", ctypes.c_int32), ("frac_bits", ctypes.c_int32), ("box", ctypes.c_double),
        ("omega_m", ctypes.c_double), ("omega_l", ctypes.c_double),
        ("c_light", ctypes.c_double), ("c_grav", ctypes.c_double),
        ("x_obs", ctypes.c_double * 3), ("shrink", ctypes.c_int32),
        ("margin", ctypes.c_int32), ("box_align", ctypes.c_int32),
        ("mg_levels", ctypes.c_int32), ("pre", ctypes.c_int32), ("post", ctypes.c_int32),
        ("coarse_sweeps", ctypes.c_int32), ("max_outer", ctypes.c_int32),
        ("tol", ctypes.c_double), ("precision", ctypes.c_int32),
        ("warm_start", ctypes.c_int32), ("n_initial", ctypes.c_int64),
        ("sort_every", ctypes.c_int32), ("sort_shift", ctypes.c_int32),
        ("solver", ctypes.c_int32), ("cycles_per_outer", ctypes.c_int32),
        ("assignment", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name == "x_obs" else v
        return out


class Particles(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p * 3), ("p", ctypes.c_void_p * 3),
                ("id", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


class Lightcone(ctypes.Structure):
    _fields_ = [("id", ctypes.c_void_p), ("a", ctypes.c_void_p), ("x", ctypes.c_void_p * 3),
                ("p", ctypes.c_void_p * 3), ("capacity", ctypes.c_int64)]


class Fields(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_void_p), ("rhs", ctypes.c_void_p), ("counts", ctypes.c_void_p)]


class StepStats(ctypes.Structure):
    _fields_ = [
        ("n_active", ctypes.c_int64), ("n_removed", ctypes.c_int64),
        ("outer_iters", ctypes.c_int32 * 2), ("vcycles", ctypes.c_int32),
        ("warm_used", ctypes.c_int32), ("res0", ctypes.c_double * 2),
        ("res", ctypes.c_double * 2), ("dtau", ctypes.c_double), ("a_half", ctypes.c_double),
        ("kappa_h2", ctypes.c_double * 2), ("r_lc", ctypes.c_double),
        ("lo", ctypes.c_int32 * 3), ("hi", ctypes.c_int32 * 3), ("periodic", ctypes.c_int32),
        ("ms", ctypes.c_float * 8), ("res_guess", ctypes.c_double * 2),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


_LIB = None


def library() -> ctypes.CDLL:
    """Load libsdpm.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1709_04703_amd.build`")
    # torch ships its own HIP runtime (same soname as ROCm's); loading it
    # first makes libsdpm bind to that one runtime instead of a second copy.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "sdpm_step_scalars": [P(Config), dbl, dbl, P(dbl)],
        "sdpm_lightcone_radius": [P(Config), dbl, P(dbl)],
        "sdpm_domain_box": [P(Config), dbl, P(i32), P(i32), P(i32)],
        "sdpm_config_default": [P(Config), i32, dbl],
        "sdpm_workspace_bytes": [P(Config), i64, P(i64)],
        "sdpm_create": [P(Config), vp, i64, vp, P(vp)],
        "sdpm_bind": [vp, P(Particles), P(Fields), i64],
        "sdpm_init_potential": [vp, dbl, P(StepStats)],
        "sdpm_step": [vp, dbl, dbl, P(StepStats)],
        "sdpm_shrink": [vp, dbl, P(i64), vp],
        "sdpm_shrink_radius": [vp, dbl, P(i64), vp],
        "sdpm_get_state": [vp, P(StepStats)],
        "sdpm_deposit": [vp],
        "sdpm_solve": [vp, dbl, dbl, P(StepStats)],
        "sdpm_interp_force": [vp, P(vp)],
        "sdpm_sort": [vp],
        "sdpm_set_warmstart_weights": [vp, vp, i64],
        "sdpm_conv3d": [i32, vp, vp, vp, i32, vp, vp, vp],
        "sdpm_conv3d_wgrad": [i32, vp, vp, vp, vp, vp, i64, vp],
        "sdpm_net_scratch_bytes": [i32, P(i64)],
        "sdpm_net_prep": [i32, vp, vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp, vp],
        "sdpm_net_forward": [i32, vp, vp, vp, vp, vp, vp],
        "sdpm_net_forward_noalloc": [i32, vp, vp, vp, vp],
        "sdpm_net_train_step": [i32, vp, vp, vp, i32, ctypes.c_float, vp, vp, ctypes.c_float, vp,
                                i64, vp, vp],
        "sdpm_record": [vp, vp, i64],
        "sdpm_record_info": [vp, P(i64), P(dbl), P(dbl), P(dbl), i64],
        "sdpm_profile": [vp, i32],
        "sdpm_profile_read": [vp, P(KernelStat), i32, P(i32)],
        "sdpm_profile_kernels": [vp, ctypes.c_char_p],
        "sdpm_destroy": [vp],
        "sdpm_set_lightcone": [vp, P(Lightcone)],
        "sdpm_lightcone_count": [vp, P(i64)],
        "sdpm_ade_sweep": [vp, dbl, i32],
        "sdpm_rb_sweeps": [i32, vp, vp, vp, ctypes.c_float, ctypes.c_float, i32, i32, vp,
                           ctypes.c_float, P(i32), vp],
        "sdpm_pk_workspace_bytes": [i32, P(i64)],
        "sdpm_power_spectrum": [P(vp), i64, dbl, i32, i32, vp, i64, vp, P(dbl), P(dbl), P(dbl),
                                P(i64)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.sdpm_last_error.argtypes = [vp]
    lib.sdpm_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


class SdpmError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {message}")
        self.code = code


def check(code: int, ctx=None) -> int:
    if code != SDPM_OK:
        msg = library().sdpm_last_error(ctx)
        raise SdpmError(code, msg.decode() if msg else "")
    return code


# ------------------------------------------------------------ host-only calls
def config_default(ng: int, box: float, **overrides) -> Config:
    cfg = Config()
    check(library().sdpm_config_default(ctypes.byref(cfg), ng, box))
    for k, v in overrides.items():
        if k == "x_obs":
            cfg.x_obs = (ctypes.c_double * 3)(*v)
        else:
            setattr(cfg, k, v)
    return cfg


def step_scalars(cfg: Config, a: float, da: float) -> dict:
    out = (ctypes.c_double * 7)()
    check(library().sdpm_step_scalars(ctypes.byref(cfg), a, da, out))
    keys = ["dtau", "a_half", "s_half", "kappa1_h2", "kappa2_h2", "r_lc_end", "c_g"]
    return dict(zip(keys, list(out)))


def lightcone_radius(cfg: Config, a: float) -> float:
    r = ctypes.c_double()
    check(library().sdpm_lightcone_radius(ctypes.byref(cfg), a, ctypes.byref(r)))
    return r.value


def domain_box(cfg: Config, r: float):
    lo, hi = (ctypes.c_int32 * 3)(), (ctypes.c_int32 * 3)()
    per = ctypes.c_int32()
    check(library().sdpm_domain_box(ctypes.byref(cfg), r, lo, hi, ctypes.byref(per)))
    return bool(per.value), np.array(list(lo)), np.array(list(hi))


def workspace_bytes(cfg: Config, capacity: int) -> int:
    b = ctypes.c_int64()
    check(library().sdpm_workspace_bytes(ctypes.byref(cfg), capacity, ctypes.byref(b)))
    return b.value


# ------------------------------------------------------- learned warm start
def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def conv3d(n, inp, w, bias, flags, mask, out):
    """One convolution layer (see sdpm_conv3d); torch device tensors."""
    check(library().sdpm_conv3d(n, _ptr(inp), _ptr(w), _ptr(bias), flags, _ptr(mask), _ptr(out),
                                _stream()))


def rb_sweeps(n, e, e_out, r, scale: float, inv_diag: float, first: bool, fused: bool,
              t_out=None, kappa_h2: float = 0.0, box=None):
    """Four red-black half sweeps on an FP32 level in colour-split storage
    (periodic, or over the frozen-exterior box (lo, hi)), and with t_out the
    red residual of the result (see sdpm_rb_sweeps); torch device tensors of
    n^3 floats (e may be None when first)."""
    bx = None
    if box is not None:
        lo, hi = box
        bx = (ctypes.c_int32 * 6)(*lo, *hi)
    check(library().sdpm_rb_sweeps(n, _ptr(e), _ptr(e_out), _ptr(r), scale, inv_diag,
                                   1 if first else 0, 1 if fused else 0, _ptr(t_out), kappa_h2,
                                   bx, _stream()))


def pk_workspace_bytes(ng: int) -> int:
    b = ctypes.c_int64()
    check(library().sdpm_pk_workspace_bytes(ng, ctypes.byref(b)))
    return b.value


def power_spectrum(x, box: float, ng: int, shot: bool = True, jing: bool = True) -> dict:
    """P(k) of positions x (a (3, n) FP64 device tensor, or three (n,)
    tensors, each in [0, box]) on an ng^3 mesh (see sdpm_power_spectrum);
    returns numpy arrays k, p, p_raw, modes over the ng/2 shells."""
    import torch
    xs = [x[d] for d in range(3)]
    for v in xs:
        if v.dtype != torch.float64 or not v.is_cuda or not v.is_contiguous():
            raise ValueError("positions must be contiguous FP64 device tensors")
    n = int(xs[0].numel())
    ws = torch.empty(pk_workspace_bytes(ng), dtype=torch.uint8, device=xs[0].device)
    nb = ng // 2
    k, p, praw = (np.zeros(nb) for _ in range(3))
    modes = np.zeros(nb, dtype=np.int64)
    arr = (ctypes.c_void_p * 3)(*(v.data_ptr() for v in xs))
    flags = (SDPM_PK_SHOT if shot else 0) | (SDPM_PK_JING if jing else 0)
    dp = ctypes.POINTER(ctypes.c_double)
    check(library().sdpm_power_spectrum(arr, n, box, ng, flags, _ptr(ws), ws.numel(), _stream(),
                                        k.ctypes.data_as(dp), p.ctypes.data_as(dp),
                                        praw.ctypes.data_as(dp),
                                        modes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    del ws
    return {"k": k, "p": p, "p_raw": praw, "modes": modes}


def net_scratch_bytes(n: int) -> int:
    b = ctypes.c_int64()
    check(library().sdpm_net_scratch_bytes(n, ctypes.byref(b)))
    return b.value


def conv3d_wgrad(n, inp, g, dw, db, scratch):
    check(library().sdpm_conv3d_wgrad(n, _ptr(inp), _ptr(g), _ptr(dw), _ptr(db), _ptr(scratch),
                                      scratch.numel() * scratch.element_size(), _stream()))


def net_prep(n, r, phi, s_r, s_phi, kappa_h2, act0):
    check(library().sdpm_net_prep(n, _ptr(r), _ptr(phi), s_r, s_phi, kappa_h2, _ptr(act0),
                                  _stream()))


def net_forward(n, params, act0, act_a, act_b, out):
    check(library().sdpm_net_forward(n, _ptr(params), _ptr(act0), _ptr(act_a), _ptr(act_b),
                                     _ptr(out), _stream()))


def net_forward_noalloc(n, params, act0, out):
    check(library().sdpm_net_forward_noalloc(n, _ptr(params), _ptr(act0), _ptr(out), _stream()))


def net_train_step(n, params, m1, m2, step, lr, act0, target, target_scale, scratch, loss):
    check(library().sdpm_net_train_step(n, _ptr(params), _ptr(m1), _ptr(m2), step, lr, _ptr(act0),
                                        _ptr(target), target_scale, _ptr(scratch),
                                        scratch.numel() * scratch.element_size(), _ptr(loss),
                                        _stream()))


# ----------------------------------------------------------------- context
class Simulation:
    """One context with torch-owned device buffers for particles, fields and
    the workspace.  Arrays: x (3, capacity) float64, p (3, capacity) float32
    (mixed) or float64 (plain FP64), ids (capacity,) int32 holding uint32
    labels, phi / rhs (ng, ng, ng) float64, counts (ng, ng, ng) int64 holding
    uint64 fixed-point masses."""

    def __init__(self, cfg: Config, capacity: int, device: str = "cuda:0"):
        import torch

        self.torch = torch
        self.cfg = cfg
        self.lib = library()
        self.device = torch.device(device)
        ng = cfg.ng
        pdt = torch.float32 if cfg.precision == SDPM_MIXED else torch.float64
        self.x = torch.zeros((3, capacity), dtype=torch.float64, device=self.device)
        self.p = torch.zeros((3, capacity), dtype=pdt, device=self.device)
        self.ids = torch.zeros((capacity,), dtype=torch.int32, device=self.device)
        self.phi = torch.zeros((ng, ng, ng), dtype=torch.float64, device=self.device)
        self.rhs = torch.zeros((ng, ng, ng), dtype=torch.float64, device=self.device)
        self.counts = torch.zeros((ng, ng, ng), dtype=torch.int64, device=self.device)
        self.ws_bytes = workspace_bytes(cfg, capacity)
        self.workspace = torch.empty((self.ws_bytes,), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.capacity = capacity
        self.n_active = 0
        ctx = ctypes.c_void_p()
        check(self.lib.sdpm_create(ctypes.byref(cfg), ctypes.c_void_p(self.workspace.data_ptr()),
                                   self.ws_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(ctx)))
        self.ctx = ctx

    # -- lifetime
    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.sdpm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, code):
        return check(code, self.ctx)

    # -- binding
    def _structs(self):
        parts = Particles()
        for d in range(3):
            parts.x[d] = self.x[d].data_ptr()
            parts.p[d] = self.p[d].data_ptr()
        parts.id = self.ids.data_ptr()
        parts.capacity = self.capacity
        fields = Fields(self.phi.data_ptr(), self.rhs.data_ptr(), self.counts.data_ptr())
        return parts, fields

    def bind(self, x, p, ids, phi=None):
        """Copy host/device arrays x (n,3), p (n,3), ids (n,) into the bound
        buffers and bind them (n active)."""
        torch = self.torch
        n = int(np.shape(x)[0])
        if n > self.capacity:
            raise ValueError("more particles than capacity")
        xt = torch.as_tensor(np.ascontiguousarray(np.asarray(x, dtype=np.float64).T))
        pt = torch.as_tensor(np.ascontiguousarray(np.asarray(p, dtype=np.float64).T))
        it = torch.as_tensor(np.asarray(ids, dtype=np.uint32).view(np.int32))
        self.x[:, :n].copy_(xt)
        self.p[:, :n].copy_(pt.to(self.p.dtype))
        self.ids[:n].copy_(it)
        if phi is not None:
            self.phi.copy_(torch.as_tensor(np.asarray(phi, dtype=np.float64)))
        else:
            self.phi.zero_()
        torch.cuda.synchronize(self.device)
        parts, fields = self._structs()
        self._check(self.lib.sdpm_bind(self.ctx, ctypes.byref(parts), ctypes.byref(fields), n))
        self.n_active = n

    # -- the path
    def init_potential(self, a: float) -> dict:
        st = StepStats()
        self._check(self.lib.sdpm_init_potential(self.ctx, a, ctypes.byref(st)))
        self.n_active = st.n_active
        return st.as_dict()

    def step(self, a: float, da: float, raise_on_error: bool = True) -> dict:
        st = StepStats()
        rc = self.lib.sdpm_step(self.ctx, a, da, ctypes.byref(st))
        self.n_active = (st.n_active if rc in (SDPM_OK, SDPM_ENOCONV, SDPM_EDOMAIN, SDPM_EFULL)
                         else self.n_active)
        if raise_on_error:
            self._check(rc)
        d = st.as_dict()
        d["rc"] = rc
        return d

    def shrink(self, a: float, removed_ids=None) -> int:
        nr = ctypes.c_int64()
        ptr = ctypes.c_void_p(removed_ids.data_ptr()) if removed_ids is not None else None
        self._check(self.lib.sdpm_shrink(self.ctx, a, ctypes.byref(nr), ptr))
        self.n_active -= nr.value
        return nr.value

    def shrink_radius(self, r: float, removed_ids=None) -> int:
        nr = ctypes.c_int64()
        ptr = ctypes.c_void_p(removed_ids.data_ptr()) if removed_ids is not None else None
        self._check(self.lib.sdpm_shrink_radius(self.ctx, r, ctypes.byref(nr), ptr))
        self.n_active -= nr.value
        return nr.value

    def state(self) -> dict:
        st = StepStats()
        self._check(self.lib.sdpm_get_state(self.ctx, ctypes.byref(st)))
        return st.as_dict()

    def deposit(self):
        self._check(self.lib.sdpm_deposit(self.ctx))

    def solve(self, kappa_h2: float, s_source: float) -> dict:
        st = StepStats()
        self._check(self.lib.sdpm_solve(self.ctx, kappa_h2, s_source, ctypes.byref(st)))
        return st.as_dict()

    def ade_sweep(self, lam: float, forward: bool = True):
        """One ADE sweep of phi in place with rhs as the source."""
        self._check(self.lib.sdpm_ade_sweep(self.ctx, lam, 1 if forward else 0))

    def sort(self):
        self._check(self.lib.sdpm_sort(self.ctx))

    def interp_force(self):
        n = self.n_active
        g = self.torch.zeros((3, max(n, 1)), dtype=self.torch.float64, device=self.device)
        arr = (ctypes.c_void_p * 3)(*(g[d].data_ptr() for d in range(3)))
        self._check(self.lib.sdpm_interp_force(self.ctx, arr))
        return g[:, :n]

    # -- lightcone output
    def set_lightcone(self, capacity: int):
        """Record removed particles at their lightcone crossing into device
        buffers of `capacity` records (capacity 0 disables)."""
        torch = self.torch
        if capacity <= 0:
            self._lc = None
            self._check(self.lib.sdpm_set_lightcone(self.ctx, None))
            return
        dev = self.device
        self._lc = dict(id=torch.zeros(capacity, dtype=torch.int32, device=dev),
                        a=torch.zeros(capacity, dtype=torch.float64, device=dev),
                        x=torch.zeros((3, capacity), dtype=torch.float64, device=dev),
                        p=torch.zeros((3, capacity), dtype=torch.float64, device=dev))
        lc = Lightcone()
        lc.id = self._lc["id"].data_ptr()
        lc.a = self._lc["a"].data_ptr()
        for d in range(3):
            lc.x[d] = self._lc["x"][d].data_ptr()
            lc.p[d] = self._lc["p"][d].data_ptr()
        lc.capacity = capacity
        self._check(self.lib.sdpm_set_lightcone(self.ctx, ctypes.byref(lc)))

    def lightcone_count(self) -> int:
        cnt = ctypes.c_int64()
        self._check(self.lib.sdpm_lightcone_count(self.ctx, ctypes.byref(cnt)))
        return cnt.value

    def lightcone_records(self):
        """(ids, a, x (n, 3), p (n, 3)) of the records written so far (host)."""
        n = self.lightcone_count()
        self.torch.cuda.synchronize(self.device)
        lc = self._lc
        return (lc["id"][:n].cpu().numpy().view(np.uint32).copy(), lc["a"][:n].cpu().numpy().copy(),
                lc["x"][:, :n].T.cpu().numpy().copy(), lc["p"][:, :n].T.cpu().numpy().copy())

    # -- learned warm start and solve recording
    def set_warmstart_weights(self, params):
        arr = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        self._check(self.lib.sdpm_set_warmstart_weights(
            self.ctx, arr.ctypes.data_as(ctypes.c_void_p), arr.size))

    def record(self, buf, max_solves: int):
        """Record up to max_solves solves into buf (torch float32 device
        tensor of at least max_solves * 3 * ng^3 entries)."""
        self._record_buf = buf
        self._check(self.lib.sdpm_record(self.ctx, _ptr(buf), max_solves))

    def record_info(self):
        cnt = ctypes.c_int64()
        self._check(self.lib.sdpm_record_info(self.ctx, ctypes.byref(cnt), None, None, None, 0))
        k = max(cnt.value, 1)
        kap, rr, rp = (ctypes.c_double * k)(), (ctypes.c_double * k)(), (ctypes.c_double * k)()
        self._check(self.lib.sdpm_record_info(self.ctx, ctypes.byref(cnt), kap, rr, rp, k))
        n = cnt.value
        return n, np.array(kap[:n]), np.array(rr[:n]), np.array(rp[:n])

    # -- tracing
    def profile(self, enable: bool = True, kernels=None):
        """Per-kernel event timing on (all kernels, or only those named in
        `kernels`, an iterable of profile names) or off; totals cleared."""
        if enable and kernels is not None:
            self._check(self.lib.sdpm_profile_kernels(self.ctx, ",".join(kernels).encode()))
        else:
            self._check(self.lib.sdpm_profile(self.ctx, 1 if enable else 0))

    def profile_read(self) -> dict:
        arr = (KernelStat * 64)()
        n = ctypes.c_int32()
        self._check(self.lib.sdpm_profile_read(self.ctx, arr, 64, ctypes.byref(n)))
        out = {}
        for k in range(n.value):
            out[arr[k].name.decode()] = dict(launches=arr[k].launches, ms=arr[k].ms,
                                             bytes=arr[k].bytes)
        return out

    # -- host copies
    def particles(self, all_particles: bool = False):
        n = self.capacity if all_particles else self.n_active
        self.torch.cuda.synchronize(self.device)
        x = self.x[:, :n].T.cpu().numpy().copy()
        p = self.p[:, :n].T.double().cpu().numpy().copy()
        ids = self.ids[:n].cpu().numpy().view(np.uint32).copy()
        return x, p, ids

    def counts_numpy(self) -> np.ndarray:
        return self.counts.cpu().numpy().view(np.uint64)

    def phi_numpy(self) -> np.ndarray:
        return self.phi.cpu().numpy()
