"""ctypes binding of liblbtp (include/lbtp.h).

Argument marshalling only: every step of the method runs in the HIP
library.  Device buffers come from torch (CUDA/HIP tensors); host arrays
(numpy) are accepted too and copied by the library.  If liblbtp.so is not
built, or there is no GPU, constructing a Solver raises at once.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbtp.so")

D2Q5, D3Q7, D2Q9 = 0, 1, 2
COEF_QUADRATIC_KR, COEF_RATIONAL = 0, 1
COLLISION_BGK, COLLISION_MRT = 0, 1
_LATTICE = {"D2Q5": D2Q5, "D3Q7": D3Q7, "D2Q9": D2Q9}
_Q = {D2Q5: 5, D3Q7: 7, D2Q9: 9}
FP32, FP16_DEV, BF16_DEV = 0, 1, 2
BC_PERIODIC, BC_DIRICHLET, BC_NOFLUX, BC_OUTFLOW = 0, 1, 2, 3
OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, EUNSTABLE, ESTATE = 0, 1, -1, -2, -3, -4, -5

_BC = {"periodic": BC_PERIODIC, "abb": BC_DIRICHLET, "dirichlet": BC_DIRICHLET,
       "bb": BC_NOFLUX, "noflux": BC_NOFLUX, "outflow": BC_OUTFLOW}
_STORAGE = {"fp32": FP32, "fp16": FP16_DEV, "bf16": BF16_DEV}


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("dx", ctypes.c_double), ("dt", ctypes.c_double),
        ("beta", ctypes.c_double), ("Ds", ctypes.c_double),
        ("mu_w", ctypes.c_double), ("mu_n", ctypes.c_double),
        ("storage", ctypes.c_int),
        ("residual_stride", ctypes.c_int),
        ("bc_f", ctypes.c_int * 6), ("bc_P", ctypes.c_double * 6),
        ("bc_g", ctypes.c_int * 6), ("bc_S", ctypes.c_double * 6),
        ("init_neq", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("coef_model", ctypes.c_int),
        ("coef", ctypes.c_double * 6),
        ("cap_B", ctypes.c_double),
        ("sweep_block", ctypes.c_int),
        ("collision", ctypes.c_int),
        ("mrt_rates", ctypes.c_double * 3),
    ]


EXPORTS = {
    "lbtp_default_params": (None, [ctypes.POINTER(Params)]),
    "lbtp_init": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_void_p)]),
    "lbtp_destroy": (None, [ctypes.c_void_p]),
    "lbtp_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "lbtp_set_fields": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4 + [ctypes.c_int]),
    "lbtp_set_sources": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 2 + [ctypes.c_int]),
    "lbtp_phase_velocities": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "lbtp_set_wall_values": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int]),
    "lbtp_set_wall_types": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int]),
    "lbtp_set_state": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4 + [ctypes.c_int]),
    "lbtp_probe_sweeps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_longlong]),
    "lbtp_update_coefficients": (ctypes.c_int, [ctypes.c_void_p]),
    "lbtp_pressure_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_longlong,
                                           ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double)]),
    "lbtp_saturation_step": (ctypes.c_int, [ctypes.c_void_p]),
    "lbtp_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_double, ctypes.c_longlong,
                                 ctypes.c_void_p]),
    "lbtp_pressure": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "lbtp_velocity": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "lbtp_grad_p": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "lbtp_saturation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "lbtp_mass": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]),
    "lbtp_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "lbtp_checkpoint_size": (ctypes.c_longlong, [ctypes.c_void_p]),
    "lbtp_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_longlong, ctypes.c_int]),
    "lbtp_put_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_longlong, ctypes.c_int]),
    "lbtp_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lbtp_copy_probe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p]),
    "lbtp_batch_init": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "lbtp_batch_destroy": (None, [ctypes.c_void_p]),
    "lbtp_batch_size": (ctypes.c_int, [ctypes.c_void_p]),
    "lbtp_batch_set_fields": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 4 + [ctypes.c_int]),
    "lbtp_batch_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 4 + [ctypes.c_int]),
    "lbtp_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_double, ctypes.c_longlong,
                                       ctypes.c_void_p]),
    "lbtp_batch_pressure": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]),
    "lbtp_batch_saturation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]),
    "lbtp_batch_velocity": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]),
    "lbtp_batch_mass": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]),
    "lbtp_batch_set_threads": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "lbtp_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "lbtp_batch_tiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "lbtp_nn_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "lbtp_nn_destroy": (None, [ctypes.c_void_p]),
    "lbtp_nn_num_params": (ctypes.c_longlong, [ctypes.c_void_p]),
    "lbtp_nn_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "lbtp_nn_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "lbtp_nn_predict": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]),
    "lbtp_nn_predict_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "lbtp_nn_loss_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_int]),
    "lbtp_nn_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int]),
}

_lib = None


def load():
    """Load liblbtp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1808_07554_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class LbtpError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {load().lbtp_strerror(code).decode()} ({code})")


def _check(code, what):
    if code < 0:
        raise LbtpError(code, what)
    return code


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("liblbtp needs a HIP device; none is visible")
    return torch


class _Arg:
    """A caller array as (pointer, on_device, keep-alive)."""

    def __init__(self, a, n, torch=None):
        if a is None:
            self.ptr, self.dev, self.keep = None, 0, None
            return
        if torch is not None and isinstance(a, torch.Tensor):
            if a.dtype != torch.float32:
                a = a.float()
            a = a.contiguous()
            if a.numel() != n:
                raise ValueError(f"expected {n} values, got {a.numel()}")
            self.dev = 1 if a.is_cuda else 0
            self.ptr, self.keep = a.data_ptr(), a
        else:
            h = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
            if h.size != n:
                raise ValueError(f"expected {n} values, got {h.size}")
            self.ptr, self.dev, self.keep = h.ctypes.data, 0, h


def _face_constant(b, lattice):
    """(condition, value) of a face rule for lbtp_params.  A mixed face
    ("links", pick, rule_a, rule_b) takes the condition and value of its
    rule that is not bounce-back; its links get their own conditions from
    link_types after lbtp_init."""
    if b[0] != "links":
        return _BC[b[0]], (float(b[1]) if len(b) > 1 else 0.0)
    if lattice != "D2Q9":
        raise ValueError("per-link conditions need D2Q9")
    rules = [r for r in (b[2], b[3]) if r[0] != "bb"]
    if len(rules) > 1 and tuple(rules[0]) != tuple(rules[1]):
        raise ValueError("a mixed face holds one condition besides bounce-back")
    return _face_constant(rules[0] if rules else b[2], lattice)


def link_types(shape, dx, face, rule, periodic_axes=()):
    """Per-link conditions of a D2Q9 face (the lbtp_set_wall_types layout)
    from a ("links", pick, rule_a, rule_b) rule: pick(x, y, z, t) is taken at
    the midpoint of each link, node - c_i dt / 2, with nodes at (j + 1/2) dx
    on walled axes and j dx on periodic ones."""
    _, pick, ra, rb = rule
    nx, ny = shape[0], shape[1]
    off = [0.0 if a in periodic_axes else 0.5 for a in range(2)]
    n_along = ny if face < 2 else nx
    along = (np.arange(n_along) + off[1 if face < 2 else 0]) * dx
    inward = (1, -1, 1, -1)[face]
    X = np.empty((n_along, 3))
    Y = np.empty((n_along, 3))
    for k, t in enumerate((0, -1, 1)):           # slots: normal, tangential -1, +1
        if face < 2:
            ex, ey = inward, t
            X[:, k] = (off[0] if face == 0 else nx - 1 + off[0]) * dx - 0.5 * ex * dx
            Y[:, k] = along - 0.5 * ey * dx
        else:
            ex, ey = t, inward
            X[:, k] = along - 0.5 * ex * dx
            Y[:, k] = (off[1] if face == 2 else ny - 1 + off[1]) * dx - 0.5 * ey * dx
    sel = np.broadcast_to(np.asarray(pick(X, Y, np.zeros_like(X), 0.0), dtype=bool), X.shape)
    return np.where(sel, _BC[ra[0]], _BC[rb[0]]).astype(np.int32).ravel()


def make_params(lattice, shape, *, beta, Ds, mu_w=1.0, mu_n=1.0, bc_f, bc_g, dx=1.0, dt=1.0, m=64,
                storage="fp32", init_neq=True, stream_ptr=None, coef=None, cap_B=0.0, sweep_block=0,
                collision=None, **_):
    """lbtp_params from keyword values.  coef: None for the quadratic relative
    permeabilities with mu_w, mu_n, or ("rational", a0, a1, c0, c1, b0, b1)
    for D_p = K (a0 + a1 S)/(b0 + b1 S), lambda_w K = K (c0 + c1 S)/(b0 + b1 S)."""
    lib = load()
    p = Params()
    lib.lbtp_default_params(ctypes.byref(p))
    p.lattice = _LATTICE[lattice]
    shape = tuple(shape) + (1,) * (3 - len(shape))
    p.nx, p.ny, p.nz = shape
    p.dx, p.dt, p.beta, p.Ds, p.mu_w, p.mu_n = dx, dt, beta, Ds, mu_w, mu_n
    p.storage = _STORAGE[storage] if isinstance(storage, str) else storage
    p.residual_stride = m
    for f, b in enumerate(bc_f):
        p.bc_f[f], p.bc_P[f] = _face_constant(b, lattice)
    for f, b in enumerate(bc_g):
        p.bc_g[f], p.bc_S[f] = _face_constant(b, lattice)
    p.init_neq = 1 if init_neq else 0
    p.stream = stream_ptr
    p.cap_B = float(cap_B)
    p.sweep_block = int(sweep_block)
    if collision is not None:
        if collision[0] != "mrt" or len(collision) != 4:
            raise ValueError(f"unknown collision {collision!r}")
        p.collision = COLLISION_MRT
        for i, v in enumerate(collision[1:]):
            p.mrt_rates[i] = float(v)
    if coef is not None:
        if coef[0] != "rational" or len(coef) != 7:
            raise ValueError(f"unknown coefficient model {coef!r}")
        p.coef_model = COEF_RATIONAL
        for i, v in enumerate(coef[1:]):
            p.coef[i] = float(v)
    return p, shape


class Batch:
    """An ensemble of realisations advanced together (lbtp_batch_*).

    members: list of parameter dicts (as produced by paper_1808_07554_amd.inputs).
    The ensemble runs on a stream of its own unless `stream` is given.
    """

    def __init__(self, members, m=64, storage="fp32", stream=None):
        self.torch = _torch()
        lib = load()
        n = len(members)
        arr = (Params * n)()
        self.shapes = []
        sptr = stream.cuda_stream if stream is not None else None
        for i, d in enumerate(members):
            d = dict(d)
            p, shape = make_params(d.pop("lattice"), d.pop("shape"), m=m, storage=storage, stream_ptr=sptr, **d)
            arr[i] = p
            self.shapes.append(shape)
        self.dim = 3 if arr[0].lattice == D3Q7 else 2
        h = ctypes.c_void_p()
        _check(lib.lbtp_batch_init(arr, n, ctypes.byref(h)), "lbtp_batch_init")
        self._h, self._lib, self.n = h, lib, n

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.lbtp_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ncell(self, i):
        s = self.shapes[i]
        return s[0] * s[1] * s[2]

    def _fshape(self, i):
        s = self.shapes[i]
        return (s[2], s[1], s[0])

    def set_fields(self, i, K, phi, Fp=None, Fs=None):
        a = [_Arg(x, self._ncell(i), self.torch) for x in (K, phi, Fp, Fs)]
        dev = {x.dev for x in a if x.ptr is not None}
        _check(self._lib.lbtp_batch_set_fields(self._h, i, *(x.ptr for x in a), dev.pop() if dev else 0),
               "lbtp_batch_set_fields")

    def set_state(self, i, P0, S0, dP0=None, dS0=None):
        n = self._ncell(i)
        a = [_Arg(P0, n, self.torch), _Arg(S0, n, self.torch), _Arg(dP0, self.dim * n, self.torch),
             _Arg(dS0, self.dim * n, self.torch)]
        dev = {x.dev for x in a if x.ptr is not None}
        _check(self._lib.lbtp_batch_set_state(self._h, i, *(x.ptr for x in a), dev.pop() if dev else 0),
               "lbtp_batch_set_state")

    def step(self, nsteps, tol, max_iters):
        its = (ctypes.c_longlong * max(1, nsteps * self.n))()
        st = _check(self._lib.lbtp_batch_step(self._h, int(nsteps), tol, int(max_iters),
                                              ctypes.cast(its, ctypes.c_void_p)), "lbtp_batch_step")
        return np.array(list(its)[: nsteps * self.n], dtype=np.int64).reshape(nsteps, self.n), st

    def _out(self, fn, i, ncomp, what):
        t = self.torch.empty(ncomp * self._ncell(i), dtype=self.torch.float32, device="cuda")
        _check(fn(self._h, i, ctypes.c_void_p(t.data_ptr()), 1), what)
        return t

    def pressure(self, i):
        return self._out(self._lib.lbtp_batch_pressure, i, 1, "lbtp_batch_pressure").view(self._fshape(i))

    def saturation(self, i):
        return self._out(self._lib.lbtp_batch_saturation, i, 1, "lbtp_batch_saturation").view(self._fshape(i))

    def velocity(self, i):
        return self._out(self._lib.lbtp_batch_velocity, i, self.dim, "lbtp_batch_velocity").view(
            (self.dim,) + self._fshape(i))

    def mass(self, i):
        m, l = ctypes.c_double(), ctypes.c_double()
        _check(self._lib.lbtp_batch_mass(self._h, i, ctypes.byref(m), ctypes.byref(l)), "lbtp_batch_mass")
        return m.value, l.value

    def set_threads(self, nt):
        _check(self._lib.lbtp_batch_set_threads(self._h, int(nt)), "lbtp_batch_set_threads")

    def autotune(self, sweeps=10):
        t = ctypes.c_int()
        _check(self._lib.lbtp_batch_autotune(self._h, int(sweeps), ctypes.byref(t)), "lbtp_batch_autotune")
        return t.value

    def tiling(self, i):
        """(waves, rows per wave, sweeps per launch) of member i's blocked tiling."""
        w, r, h = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self._lib.lbtp_batch_tiling(self._h, int(i), ctypes.byref(w), ctypes.byref(r), ctypes.byref(h)),
               "lbtp_batch_tiling")
        return w.value, r.value, h.value


def _ptr(t):
    """Device pointer of a tensor, or NULL for None."""
    return ctypes.c_void_p(None if t is None else t.data_ptr())


class WarmStartNet:
    """The learned warm start (include/lbtp_nn.h).  Fields are [N, H, W]
    float32 torch tensors on the device (or numpy arrays)."""

    def __init__(self, base=32, levels=4, scale=3.2, stream=None):
        self.torch = _torch()
        lib = load()
        s = stream if stream is not None else self.torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib.lbtp_nn_create(int(base), int(levels), float(scale), ctypes.c_void_p(s.cuda_stream),
                                  ctypes.byref(h)), "lbtp_nn_create")
        self._h, self._lib = h, lib
        self.base, self.levels, self.scale = base, levels, scale
        self.n_params = lib.lbtp_nn_num_params(h)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.lbtp_nn_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device="cuda", dtype=t.float32).contiguous()
        return t.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).cuda()

    def set_params(self, theta):
        th = self._dev(theta).ravel()
        assert th.numel() == self.n_params
        _check(self._lib.lbtp_nn_set_params(self._h, ctypes.c_void_p(th.data_ptr()), 1), "lbtp_nn_set_params")

    def get_params(self):
        th = self.torch.empty(self.n_params, dtype=self.torch.float32, device="cuda")
        _check(self._lib.lbtp_nn_get_params(self._h, ctypes.c_void_p(th.data_ptr()), 1), "lbtp_nn_get_params")
        return th

    def predict(self, lnK, S, factor=1):
        """Initial pressure [n, h, w]; factor > 1 runs the network on the grid
        coarsened by that factor and interpolates its deviation back."""
        lnK, S = self._dev(lnK), self._dev(S)
        n, h, w = lnK.shape
        P = self.torch.empty_like(lnK)
        _check(self._lib.lbtp_nn_predict(self._h, ctypes.c_void_p(lnK.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                                         n, h, w, int(factor), ctypes.c_void_p(P.data_ptr()), 1), "lbtp_nn_predict")
        return P

    def predict_noalloc(self, lnK, S, P, factor=1):
        """lbtp_nn_predict_noalloc: like predict, into the caller's device
        tensor P [n, h, w]; lnK, S and P must be contiguous float32 tensors on
        the device (the library allocates nothing)."""
        t = self.torch
        for a in (lnK, S, P):
            if not (isinstance(a, t.Tensor) and a.is_cuda and a.dtype == t.float32 and a.is_contiguous()):
                raise ValueError("predict_noalloc takes contiguous float32 device tensors")
        n, h, w = lnK.shape
        if tuple(S.shape) != (n, h, w) or tuple(P.shape) != (n, h, w):
            raise ValueError("lnK, S and P must have one shape")
        _check(self._lib.lbtp_nn_predict_noalloc(self._h, ctypes.c_void_p(lnK.data_ptr()),
                                                 ctypes.c_void_p(S.data_ptr()), n, h, w, int(factor),
                                                 ctypes.c_void_p(P.data_ptr())), "lbtp_nn_predict_noalloc")
        return P

    def _weights(self, weight):
        return None if weight is None else self._dev(weight)

    def loss_grad(self, lnK, S, P, weight=None):
        """Weighted MSE (weight: one per sample or None) and its gradient."""
        lnK, S, P, wt = self._dev(lnK), self._dev(S), self._dev(P), self._weights(weight)
        n, h, w = lnK.shape
        g = self.torch.empty(self.n_params, dtype=self.torch.float32, device="cuda")
        loss = ctypes.c_double()
        _check(self._lib.lbtp_nn_loss_grad(self._h, ctypes.c_void_p(lnK.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                                           ctypes.c_void_p(P.data_ptr()), _ptr(wt), n, h, w, ctypes.byref(loss),
                                           ctypes.c_void_p(g.data_ptr()), 1), "lbtp_nn_loss_grad")
        return loss.value, g

    def train_step(self, lnK, S, P, lr, weight=None):
        lnK, S, P, wt = self._dev(lnK), self._dev(S), self._dev(P), self._weights(weight)
        n, h, w = lnK.shape
        loss = ctypes.c_double()
        _check(self._lib.lbtp_nn_train_step(self._h, ctypes.c_void_p(lnK.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                                            ctypes.c_void_p(P.data_ptr()), _ptr(wt), n, h, w, float(lr),
                                            ctypes.byref(loss), 1), "lbtp_nn_train_step")
        return loss.value


class Solver:
    """One realisation on the GPU.  Same calls as the C ABI.

    bc_f / bc_g: per face (-x, +x, -y, +y[, -z, +z]) a tuple ("periodic",),
    ("abb", value), ("bb",) or ("outflow",); on D2Q9 also
    ("links", pick, rule_a, rule_b), a face whose links take rule_a where
    pick(x, y, z, t) holds at the link midpoint and rule_b elsewhere (one of
    the two bounce-back), passed to lbtp_set_wall_types.
    """

    def __init__(self, lattice, shape, *, beta, Ds, mu_w=1.0, mu_n=1.0, bc_f, bc_g, dx=1.0, dt=1.0, m=64,
                 storage="fp32", init_neq=True, stream=None, coef=None, cap_B=0.0, sweep_block=0,
                 collision=None, **_):
        self.torch = _torch()
        lib = load()
        if stream is None:
            stream = self.torch.cuda.current_stream()
        self.stream = stream
        p, shape = make_params(lattice, shape, beta=beta, Ds=Ds, mu_w=mu_w, mu_n=mu_n, bc_f=bc_f, bc_g=bc_g,
                               dx=dx, dt=dt, m=m, storage=storage, init_neq=init_neq,
                               stream_ptr=stream.cuda_stream, coef=coef, cap_B=cap_B, sweep_block=sweep_block,
                               collision=collision)
        self.params = p
        self.dim = 3 if p.lattice == D3Q7 else 2
        self.Q = _Q[p.lattice]
        self.shape = shape
        self.ncell = shape[0] * shape[1] * shape[2]
        h = ctypes.c_void_p()
        _check(lib.lbtp_init(ctypes.byref(p), ctypes.byref(h)), "lbtp_init")
        self._h = h
        self._lib = lib
        periodic = tuple(a for a in range(self.dim) if bc_f[2 * a][0] == "periodic")
        for face in range(len(bc_f)):
            tf, tg = (link_types(shape, dx, face, b[face], periodic) if b[face][0] == "links" else None
                      for b in (bc_f, bc_g))
            if tf is not None or tg is not None:
                self.set_wall_types(face, tf, tg)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.lbtp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- helpers
    def _arg(self, a, n=None):
        return _Arg(a, self.ncell if n is None else n, self.torch)

    def _both(self, *args):
        dev = {a.dev for a in args if a.ptr is not None}
        if len(dev) > 1:
            raise ValueError("mix of host and device arrays in one call")
        return dev.pop() if dev else 0

    def _empty(self, n):
        return self.torch.empty(n, dtype=self.torch.float32, device="cuda")

    def _fshape(self):
        return (self.shape[2], self.shape[1], self.shape[0])

    # ------------------------------------------------------------------ calls
    def set_fields(self, K, phi, Fp=None, Fs=None):
        a = [self._arg(x) for x in (K, phi, Fp, Fs)]
        _check(self._lib.lbtp_set_fields(self._h, *(x.ptr for x in a), self._both(*a)), "lbtp_set_fields")

    def set_sources(self, Fp=None, Fs=None):
        a = [self._arg(x) for x in (Fp, Fs)]
        _check(self._lib.lbtp_set_sources(self._h, *(x.ptr for x in a), self._both(*a)), "lbtp_set_sources")

    def set_wall_values(self, face, P=None, S=None):
        """Per-link Dirichlet data of one face (lbtp_set_wall_values): P and / or
        S at the midpoints of the links crossing the face (L per face node)."""
        n = self.ncell // self.shape[face // 2]
        n *= 3 if self.params.lattice == D2Q9 else 1
        a, b = self._arg(P, n), self._arg(S, n)
        _check(self._lib.lbtp_set_wall_values(self._h, int(face), a.ptr, b.ptr, self._both(a, b)),
               "lbtp_set_wall_values")

    def set_wall_types(self, face, f=None, g=None):
        """Per-link conditions of one D2Q9 face (lbtp_set_wall_types): int
        arrays of lbtp_bc values, three per face node, or None to keep."""
        n = 3 * (self.shape[1] if face < 2 else self.shape[0])
        arrs = []
        for a in (f, g):
            if a is None:
                arrs.append(None)
                continue
            a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
            if a.size != n:
                raise ValueError(f"expected {n} values, got {a.size}")
            arrs.append(a)
        ptrs = [None if a is None else a.ctypes.data for a in arrs]
        _check(self._lib.lbtp_set_wall_types(self._h, int(face), ptrs[0], ptrs[1], 0), "lbtp_set_wall_types")

    def set_state(self, P0, S0, dP0=None, dS0=None):
        a = [self._arg(P0), self._arg(S0), self._arg(dP0, self.dim * self.ncell),
             self._arg(dS0, self.dim * self.ncell)]
        _check(self._lib.lbtp_set_state(self._h, *(x.ptr for x in a), self._both(*a)), "lbtp_set_state")

    def update_coefficients(self):
        _check(self._lib.lbtp_update_coefficients(self._h), "lbtp_update_coefficients")

    def pressure_solve(self, tol, max_iters):
        it, r = ctypes.c_longlong(), ctypes.c_double()
        st = _check(self._lib.lbtp_pressure_solve(self._h, tol, int(max_iters), ctypes.byref(it), ctypes.byref(r)),
                    "lbtp_pressure_solve")
        return it.value, r.value, st

    def saturation_step(self):
        _check(self._lib.lbtp_saturation_step(self._h), "lbtp_saturation_step")

    def probe_sweeps(self, launches):
        """lbtp_probe_sweeps: `launches` back-to-back launches of the plain
        pressure sweep (timing aid); returns the sweeps per launch."""
        return _check(self._lib.lbtp_probe_sweeps(self._h, int(launches)), "lbtp_probe_sweeps")

    def step(self, nsteps, tol, max_iters):
        its = (ctypes.c_longlong * max(1, nsteps))()
        st = _check(self._lib.lbtp_step(self._h, int(nsteps), tol, int(max_iters), ctypes.cast(its, ctypes.c_void_p)),
                    "lbtp_step")
        return list(its)[:nsteps], st

    def _out(self, fn, ncomp, what):
        t = self._empty(ncomp * self.ncell)
        _check(fn(self._h, ctypes.c_void_p(t.data_ptr()), 1), what)
        return t

    def pressure(self):
        return self._out(self._lib.lbtp_pressure, 1, "lbtp_pressure").view(self._fshape())

    def saturation(self):
        return self._out(self._lib.lbtp_saturation, 1, "lbtp_saturation").view(self._fshape())

    def velocity(self):
        return self._out(self._lib.lbtp_velocity, self.dim, "lbtp_velocity").view((self.dim,) + self._fshape())

    def grad_p(self):
        return self._out(self._lib.lbtp_grad_p, self.dim, "lbtp_grad_p").view((self.dim,) + self._fshape())

    def mass(self):
        m, l = ctypes.c_double(), ctypes.c_double()
        _check(self._lib.lbtp_mass(self._h, ctypes.byref(m), ctypes.byref(l)), "lbtp_mass")
        return m.value, l.value

    def phase_velocities(self):
        """(u_w, u_n) of eq. 2-12 / 2-13, each (dim, nz, ny, nx)."""
        uw = self._empty(self.dim * self.ncell)
        un = self._empty(self.dim * self.ncell)
        _check(self._lib.lbtp_phase_velocities(self._h, ctypes.c_void_p(uw.data_ptr()),
                                               ctypes.c_void_p(un.data_ptr()), 1), "lbtp_phase_velocities")
        return uw.view((self.dim,) + self._fshape()), un.view((self.dim,) + self._fshape())

    def populations(self):
        """Pre-collision populations (float32): f_1..f_{Q-1} and g_0..g_{Q-1}."""
        f = self._empty((self.Q - 1) * self.ncell)
        g = self._empty(self.Q * self.ncell)
        _check(self._lib.lbtp_populations(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()), 1),
               "lbtp_populations")
        return f.view((self.Q - 1,) + self._fshape()), g.view((self.Q,) + self._fshape())

    def get_state(self):
        """Opaque checkpoint image (uint8 device tensor)."""
        n = self._lib.lbtp_checkpoint_size(self._h)
        _check(n, "lbtp_checkpoint_size")
        buf = self.torch.empty(n, dtype=self.torch.uint8, device="cuda")
        _check(self._lib.lbtp_get_state(self._h, ctypes.c_void_p(buf.data_ptr()), n, 1), "lbtp_get_state")
        return buf

    def put_state(self, buf):
        if isinstance(buf, self.torch.Tensor):
            buf = buf.contiguous()
            _check(self._lib.lbtp_put_state(self._h, ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                            1 if buf.is_cuda else 0), "lbtp_put_state")
        else:
            h = np.ascontiguousarray(np.frombuffer(bytes(buf), dtype=np.uint8))
            _check(self._lib.lbtp_put_state(self._h, ctypes.c_void_p(h.ctypes.data), h.size, 0), "lbtp_put_state")


def from_problem(params, **kw):
    """Solver from a plain parameter dict (as produced by paper_1808_07554_amd.inputs)."""
    d = dict(params)
    d.update(kw)
    return Solver(d.pop("lattice"), d.pop("shape"), **d)
