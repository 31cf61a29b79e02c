"""Python binding of librs (include/rs.h): argument marshalling only.

Every step of the reduced-Newton path runs in the HIP library; this module
checks tensor placement, dtype and contiguity, passes device pointers and the
current HIP stream, and raises on any error code.  It fails loudly when the
library has not been built or no GPU is present; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # imported before librs so both share one HIP runtime

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librs.so")

RS_OK, RS_ERR_ARG, RS_ERR_HIP, RS_ERR_OOM, RS_ERR_STATE, RS_ERR_UNSUPPORTED = 0, 1, 2, 3, 4, 5
CONVERGED, NOT_DESCENT, LS_MAX, ITER_MAX, NONFINITE, RUNNING = 0, 1, 2, 3, 4, -1
PREC_F64, PREC_F32, PREC_BF16 = 0, 1, 2
HESS_EXACT, ELASTIC_ONLY, ENERGY_ONLY, GRAD_REVERSE, ELEM_PSD, DEBUG_ELEM_HESS = 1, 2, 4, 8, 16, 32
# rs_solve_opts.hess values
HESS_GN, HESS_EXACT_OPT, HESS_GN_ELEM_PSD, HESS_EXACT_ELEM_PSD = 0, 1, 2, 3
PROJ_CLAMP, PROJ_ABS, PROJ_NONE = 0, 1, 2

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class _Mesh(C.Structure):
    _fields_ = [("nv", C.c_int32), ("ne", C.c_int32), ("X", _dp), ("tets", _ip),
                ("pinned", C.POINTER(C.c_uint8))]


class _Material(C.Structure):
    _fields_ = [("young", C.c_double), ("poisson", C.c_double), ("density", C.c_double),
                ("gravity", C.c_double * 3)]


class _Decoder(C.Structure):
    _fields_ = [("r", C.c_int32), ("n_hidden", C.c_int32), ("width", C.c_int32),
                ("n_out", C.c_int32), ("W", C.POINTER(_dp)), ("b", C.POINTER(_dp))]


class _Cubature(C.Structure):
    _fields_ = [("n", C.c_int32), ("elem", _ip), ("weight", _dp)]


class _Constraints(C.Structure):
    _fields_ = [("n_target", C.c_int32), ("target_vtx", _ip), ("k_c", C.c_double),
                ("n_force", C.c_int32), ("force_vtx", _ip),
                ("n_contact", C.c_int32), ("contact_vtx", _ip), ("k_ground", C.c_double),
                ("ground_y", C.c_double)]


class _Mlp(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_hidden", C.c_int32), ("width", C.c_int32), ("n_out", C.c_int32),
                ("W", C.POINTER(_dp)), ("b", C.POINTER(_dp))]


class _Load(C.Structure):
    _fields_ = [("targets", C.c_void_p), ("force", C.c_void_p), ("qbar", C.c_void_p), ("dt", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("ls_max", C.c_int32), ("c1", C.c_double),
                ("shrink", C.c_double), ("rel_tol", C.c_double), ("abs_tol", C.c_double),
                ("hess", C.c_int32), ("proj", C.c_int32), ("eig_floor", C.c_double), ("window", C.c_int32)]


class LbfgsOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("ls_max", C.c_int32), ("history", C.c_int32), ("c1", C.c_double),
                ("shrink", C.c_double), ("rel_tol", C.c_double), ("abs_tol", C.c_double), ("window", C.c_int32)]


class FullOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("ls_max", C.c_int32), ("cg_max", C.c_int32), ("c1", C.c_double),
                ("shrink", C.c_double), ("rel_tol", C.c_double), ("abs_tol", C.c_double),
                ("eta_min", C.c_double), ("eta_max", C.c_double)]


MAX_HISTORY = 16


class Info(C.Structure):
    _fields_ = [("prec", C.c_int32), ("r", C.c_int32), ("n_hidden", C.c_int32),
                ("width", C.c_int32), ("nv", C.c_int32), ("ne", C.c_int32),
                ("n_cub", C.c_int32), ("n_target", C.c_int32), ("n_force", C.c_int32),
                ("rows", C.c_int32), ("rows_pad", C.c_int32), ("max_batch", C.c_int32)]


# every symbol include/rs.h declares
SYMBOLS = ["rs_default_opts", "rs_default_lbfgs_opts", "rs_create", "rs_destroy", "rs_set_decoder",
           "rs_get_info", "rs_decode", "rs_energy_grad_hess", "rs_newton_solve", "rs_lbfgs_solve",
           "rs_lipschitz_loss", "rs_last_error", "rs_profile", "rs_profile_get", "rs_param_count",
           "rs_energy_param_grad", "rs_set_elem_hess_dump", "rs_set_decoder_device", "rs_lipschitz_param_grad",
           "rs_lipschitz_param_grad_noalloc", "rs_trainer_create", "rs_trainer_destroy", "rs_trainer_param_count",
           "rs_trainer_params", "rs_trainer_encode", "rs_trainer_grad", "rs_trainer_adam",
           "rs_default_full_opts", "rs_full_solve", "rs_pca", "rs_simulate", "rs_newton_solve_async",
           "rs_set_fused"]

_lib = None


def load_library():
    """Load librs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.rs_last_error.restype = C.c_char_p
        L.rs_last_error.argtypes = [C.c_void_p]
        for name in SYMBOLS:
            getattr(L, name)
        L.rs_create.argtypes = [C.POINTER(_Mesh), C.POINTER(_Material), C.POINTER(_Decoder),
                                C.POINTER(_Cubature), C.POINTER(_Constraints), C.c_int32, C.c_int32,
                                C.POINTER(C.c_void_p)]
        L.rs_destroy.argtypes = [C.c_void_p]
        L.rs_set_decoder.argtypes = [C.c_void_p, C.POINTER(_Decoder)]
        L.rs_get_info.argtypes = [C.c_void_p, C.POINTER(Info)]
        L.rs_decode.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.rs_energy_grad_hess.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(_Load), C.c_uint32,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.rs_newton_solve.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(_Load),
                                      C.POINTER(SolveOpts), C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p]
        L.rs_newton_solve_async.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(_Load),
                                            C.POINTER(SolveOpts), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p]
        L.rs_lbfgs_solve.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(_Load),
                                     C.POINTER(LbfgsOpts), C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]
        L.rs_lipschitz_loss.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.rs_param_count.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.rs_energy_param_grad.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(_Load), C.c_uint32,
                                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.rs_set_elem_hess_dump.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
        L.rs_set_fused.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
        L.rs_set_decoder_device.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
        L.rs_lipschitz_param_grad.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.c_void_p, C.c_void_p]
        L.rs_lipschitz_param_grad_noalloc.argtypes = L.rs_lipschitz_param_grad.argtypes
        L.rs_trainer_create.argtypes = [C.c_void_p, C.POINTER(_Mlp), C.POINTER(_Decoder), C.c_int32,
                                        C.POINTER(C.c_void_p)]
        L.rs_trainer_destroy.argtypes = [C.c_void_p]
        L.rs_trainer_param_count.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.rs_trainer_params.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.rs_trainer_encode.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.rs_trainer_grad.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.rs_trainer_adam.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_void_p]
        L.rs_default_full_opts.argtypes = [C.POINTER(FullOpts)]
        L.rs_simulate.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(_Load), C.c_int32,
                                  C.c_double, C.POINTER(SolveOpts), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.rs_pca.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_void_p]
        L.rs_full_solve.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(_Load), C.POINTER(FullOpts),
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.rs_profile.argtypes = [C.c_void_p, C.c_int32, C.c_uint32]
        L.rs_profile_get.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_char_p, C.c_int32,
                                     C.POINTER(C.c_int32), _dp, _dp, _dp]
        L.rs_default_opts.argtypes = [C.POINTER(SolveOpts)]
        _lib = L
    return _lib


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    load_library().rs_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_lbfgs_opts(**kw) -> LbfgsOpts:
    o = LbfgsOpts()
    load_library().rs_default_lbfgs_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_full_opts(**kw) -> FullOpts:
    o = FullOpts()
    load_library().rs_default_full_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, shape=None, name="tensor"):
    """Check a caller tensor: on the GPU, given dtype, contiguous (and shape)."""
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


class Context:
    """One reduced problem on the current GPU (owns an rs_ctx)."""

    def __init__(self, problem, prec: int = PREC_F64, max_batch: int = 1024):
        if not torch.cuda.is_available():
            raise RuntimeError("librs needs a HIP GPU; none is available")
        L = load_library()
        p = problem
        self.p = p
        self.r = p.r
        self.prec = prec
        self.tdtype = torch.float64 if prec == PREC_F64 else torch.float32
        self.nv, self.n = p.X.shape[0], 3 * p.X.shape[0]
        self.nt, self.nf = len(p.target_vtx), len(p.force_vtx)
        keep = []

        def f64(a):
            a = np.ascontiguousarray(a, dtype=np.float64); keep.append(a); return a

        def i32(a):
            a = np.ascontiguousarray(a, dtype=np.int32); keep.append(a); return a

        X, tets = f64(p.X), i32(p.tets)
        pinned = np.ascontiguousarray(p.pinned, dtype=np.uint8); keep.append(pinned)
        mesh = _Mesh(X.shape[0], tets.shape[0], X.ctypes.data_as(_dp), tets.ctypes.data_as(_ip),
                     pinned.ctypes.data_as(C.POINTER(C.c_uint8)))
        mat = _Material(p.young, p.poisson, p.density, (C.c_double * 3)(*[float(v) for v in p.gravity]))
        dec = self._decoder_struct(p.Ws, p.bs, keep)
        ce, cw = i32(p.cub_elem), f64(p.cub_w)
        cub = _Cubature(len(ce), ce.ctypes.data_as(_ip), cw.ctypes.data_as(_dp))
        tv, fv = i32(p.target_vtx), i32(p.force_vtx)
        cv = i32(getattr(p, "contact_vtx", np.zeros(0, np.int32)))
        con = _Constraints(len(tv), tv.ctypes.data_as(_ip), p.k_c, len(fv), fv.ctypes.data_as(_ip),
                           len(cv), cv.ctypes.data_as(_ip), float(getattr(p, "k_ground", 0.0)),
                           float(getattr(p, "ground_y", 0.0)))
        ctx = C.c_void_p()
        rc = L.rs_create(C.byref(mesh), C.byref(mat), C.byref(dec), C.byref(cub), C.byref(con),
                         prec, max_batch, C.byref(ctx))
        if rc != RS_OK:
            raise RuntimeError(f"rs_create failed with code {rc}")
        self.ctx = ctx
        self.max_batch = max_batch
        self.device = torch.device("cuda", torch.cuda.current_device())

    def _decoder_struct(self, Ws, bs, keep):
        Ws = [np.ascontiguousarray(W, dtype=np.float64) for W in Ws]
        bs = [np.ascontiguousarray(b, dtype=np.float64) for b in bs]
        keep.extend(Ws); keep.extend(bs)
        Wp = (_dp * len(Ws))(*[W.ctypes.data_as(_dp) for W in Ws])
        bp = (_dp * len(bs))(*[b.ctypes.data_as(_dp) for b in bs])
        keep.extend([Wp, bp])
        width = Ws[0].shape[0] if len(Ws) > 1 else 0
        return _Decoder(Ws[0].shape[1], len(Ws) - 1, width, Ws[-1].shape[0],
                        C.cast(Wp, C.POINTER(_dp)), C.cast(bp, C.POINTER(_dp)))

    def __del__(self):
        if getattr(self, "ctx", None) is not None and _lib is not None:
            _lib.rs_destroy(self.ctx)
            self.ctx = None

    def _check(self, rc, what):
        if rc != RS_OK:
            msg = load_library().rs_last_error(self.ctx)
            raise RuntimeError(f"{what} failed (code {rc}): {msg.decode() if msg else ''}")

    def info(self) -> Info:
        i = Info()
        self._check(load_library().rs_get_info(self.ctx, C.byref(i)), "rs_get_info")
        return i

    def set_decoder(self, Ws, bs):
        keep = []
        dec = self._decoder_struct(Ws, bs, keep)
        self._check(load_library().rs_set_decoder(self.ctx, C.byref(dec)), "rs_set_decoder")

    def param_shapes(self):
        """(W, b) shapes of every decoder layer, output layer last (the packed gradient's order)."""
        dims = [self.r] + list(self.p.hidden) + [self.n]
        return [((dims[l + 1], dims[l]), (dims[l + 1],)) for l in range(len(dims) - 1)]

    def param_count(self) -> int:
        n = C.c_int64()
        self._check(load_library().rs_param_count(self.ctx, C.byref(n)), "rs_param_count")
        return n.value

    def unpack_params(self, flat):
        """Views of a packed parameter vector as [(W, b), ...], output layer last."""
        out, off = [], 0
        for ws, bs in self.param_shapes():
            nw, nb = ws[0] * ws[1], bs[0]
            out.append((flat[off:off + nw].view(*ws), flat[off + nw:off + nw + nb]))
            off += nw + nb
        return out

    def set_decoder_flat(self, theta):
        """Load the decoder from a packed parameter vector: a float32 or float64
        device tensor is loaded on the GPU (stream-ordered), anything else is
        copied to the host and loaded from there."""
        if isinstance(theta, torch.Tensor) and theta.is_cuda:
            self.set_decoder_device(theta)
            return
        parts = self.unpack_params(torch.as_tensor(theta).detach().to("cpu", torch.float64))
        self.set_decoder([W.numpy() for W, _ in parts], [b.numpy() for _, b in parts])

    def set_decoder_device(self, theta):
        """Load the decoder from a packed float32/float64 device tensor (rs_set_decoder_device)."""
        if theta.dtype not in (torch.float32, torch.float64):
            raise TypeError("theta must be float32 or float64")
        _dev(theta, theta.dtype, (self.param_count(),), "theta")
        self._check(load_library().rs_set_decoder_device(self.ctx, _ptr(theta), int(theta.dtype == torch.float64),
                                                         _stream()), "rs_set_decoder_device")

    def lipschitz_param_grad(self, z1, z2, out=None, noalloc=False):
        """(loss (1), grad): the Lipschitz loss over the pairs (z1_b, z2_b) and its
        gradient with respect to the packed decoder parameters (float64 device tensors).
        `out` may pass preallocated (loss, grad); noalloc=True calls the variant whose
        workspace is the library's static device array."""
        B = z1.shape[0]
        _dev(z1, torch.float64, (B, self.r), "z1")
        _dev(z2, torch.float64, (B, self.r), "z2")
        if out is None:
            loss = torch.empty(1, dtype=torch.float64, device=z1.device)
            grad = torch.empty(self.param_count(), dtype=torch.float64, device=z1.device)
        else:
            loss, grad = out
            _dev(loss, torch.float64, (1,), "loss")
            _dev(grad, torch.float64, (self.param_count(),), "grad")
        fn = "rs_lipschitz_param_grad_noalloc" if noalloc else "rs_lipschitz_param_grad"
        self._check(getattr(load_library(), fn)(self.ctx, B, _ptr(z1), _ptr(z2), _ptr(loss), _ptr(grad), _stream()),
                    fn)
        return loss, grad

    def energy_param_grad(self, z, targets=None, force=None, flags=0, want_E=True, want_g=True):
        """(E (B), g = dE/dz (B x r), grad) with grad the packed gradient of sum_b E(z_b)
        with respect to the decoder parameters (float64 device tensors; E, g may be None)."""
        B = z.shape[0]
        _dev(z, torch.float64, (B, self.r), "z")
        ld, _keep = self._load(B, targets, force)
        E = torch.empty(B, dtype=torch.float64, device=z.device) if want_E else None
        g = torch.empty((B, self.r), dtype=torch.float64, device=z.device) if want_g else None
        grad = torch.empty(self.param_count(), dtype=torch.float64, device=z.device)
        self._check(load_library().rs_energy_param_grad(self.ctx, B, _ptr(z), C.byref(ld), flags, _ptr(E), _ptr(g),
                                                        _ptr(grad), _stream()), "rs_energy_param_grad")
        return E, g, grad

    def _load(self, B, targets, force, qbar=None, dt=0.0):
        t = _dev(targets, torch.float64, (B, self.nt, 3), "targets")
        f = _dev(force, torch.float64, (B, 3), "force")
        q = _dev(qbar, torch.float64, (B, self.nv, 3), "qbar")
        return _Load(t.data_ptr() if t is not None else None, f.data_ptr() if f is not None else None,
                     q.data_ptr() if q is not None else None, float(dt)), (t, f, q)

    def decode(self, z, want_x=True, want_J=True):
        B = z.shape[0]
        _dev(z, torch.float64, (B, self.r), "z")
        x = torch.empty((B, self.nv, 3), dtype=self.tdtype, device=z.device) if want_x else None
        J = torch.empty((B, self.n, self.r), dtype=self.tdtype, device=z.device) if want_J else None
        self._check(load_library().rs_decode(self.ctx, B, _ptr(z), _ptr(x), _ptr(J), _stream()), "rs_decode")
        return x, J

    def energy_grad_hess(self, z, targets=None, force=None, flags=HESS_EXACT, qbar=None, dt=0.0):
        B = z.shape[0]
        _dev(z, torch.float64, (B, self.r), "z")
        ld, _keep = self._load(B, targets, force, qbar, dt)
        E = torch.empty(B, dtype=torch.float64, device=z.device)
        eonly = bool(flags & ENERGY_ONLY)
        g = None if eonly else torch.empty((B, self.r), dtype=torch.float64, device=z.device)
        H = None if eonly or (flags & GRAD_REVERSE) else torch.empty((B, self.r, self.r), dtype=torch.float64,
                                                                         device=z.device)
        self._check(load_library().rs_energy_grad_hess(self.ctx, B, _ptr(z), C.byref(ld), flags, _ptr(E),
                                                       _ptr(g), _ptr(H), _stream()), "rs_energy_grad_hess")
        return E, g, H

    def set_elem_hess_dump(self, He):
        """Register (He: float64 device tensor, (items, n_cub, 12, 12)) or clear (None) the
        destination of RS_DEBUG_ELEM_HESS."""
        if He is None:
            self._dump = None
            self._check(load_library().rs_set_elem_hess_dump(self.ctx, None, 0), "rs_set_elem_hess_dump")
            return
        _dev(He, torch.float64, None, "He")
        if He.dim() != 4 or tuple(He.shape[1:]) != (len(self.p.cub_elem), 12, 12):
            raise ValueError("He must have shape (items, n_cub, 12, 12)")
        self._dump = He
        self._check(load_library().rs_set_elem_hess_dump(self.ctx, _ptr(He), He.shape[0]), "rs_set_elem_hess_dump")

    def set_fused(self, on=True):
        """Form the rows of J_R and run the element physics in one kernel (True) or in two kernels
        with J_R through device memory (False); the default is True in BF16 contexts and False in
        float32 ones.  Returns whether the fused kernel applies to this context (float32 or BF16,
        r = 16, last hidden width <= 128)."""
        applies = C.c_int32(0)
        self._check(load_library().rs_set_fused(self.ctx, 1 if on else 0, C.byref(applies)), "rs_set_fused")
        return bool(applies.value)

    def newton_solve(self, z0, targets=None, force=None, opts: SolveOpts | None = None, out=None, qbar=None,
                     dt=0.0, super_steps=None):
        """z0 (B x r) float64 on the GPU; returns dict of device tensors.
        `out` may pass preallocated (z, iters, status, relgrad, E) tensors; qbar
        (B x nv x 3) and dt > 0 make it one implicit-Euler step.  With
        super_steps, the stream-ordered solve (rs_newton_solve_async): exactly
        that many super-steps, no host synchronisation, unfinished items left
        with status RUNNING."""
        if super_steps is not None:
            return self._solve("rs_newton_solve_async", z0, targets, force, opts or default_opts(), out, qbar, dt,
                               extra=(int(super_steps),))
        return self._solve("rs_newton_solve", z0, targets, force, opts or default_opts(), out, qbar, dt)

    def lbfgs_solve(self, z0, targets=None, force=None, opts: LbfgsOpts | None = None, out=None):
        """As newton_solve, with the L-BFGS solver."""
        return self._solve("rs_lbfgs_solve", z0, targets, force, opts or default_lbfgs_opts(), out)

    def _solve(self, fn, z0, targets, force, o, out, qbar=None, dt=0.0, extra=()):
        B = z0.shape[0]
        _dev(z0, torch.float64, (B, self.r), "z0")
        ld, _keep = self._load(B, targets, force, qbar, dt)
        if out is None:
            z = z0.clone()
            iters = torch.empty(B, dtype=torch.int32, device=z0.device)
            status = torch.empty(B, dtype=torch.int32, device=z0.device)
            relg = torch.empty(B, dtype=torch.float64, device=z0.device)
            E = torch.empty(B, dtype=torch.float64, device=z0.device)
        else:
            z, iters, status, relg, E = out
            z.copy_(z0)
        self._check(getattr(load_library(), fn)(self.ctx, B, _ptr(z), C.byref(ld), C.byref(o), *extra, _ptr(iters),
                                                _ptr(status), _ptr(relg), _ptr(E), _stream()), fn)
        return dict(z=z, iters=iters, status=status, relgrad=relg, E=E)

    def simulate(self, z0, steps, dt, v0=None, targets=None, force=None, opts: SolveOpts | None = None,
                 want_traj=True):
        """Implicit-Euler simulation of B items (rs_simulate): dict of device tensors
        z (last step), iters and failed per item, traj (steps x B x r) when wanted."""
        B = z0.shape[0]
        _dev(z0, torch.float64, (B, self.r), "z0")
        _dev(v0, torch.float64, (B, self.nv, 3), "v0")
        ld, _keep = self._load(B, targets, force)
        z = z0.clone()
        dev = z0.device
        iters = torch.empty(B, dtype=torch.int32, device=dev)
        failed = torch.empty(B, dtype=torch.int32, device=dev)
        traj = torch.empty((steps, B, self.r), dtype=torch.float64, device=dev) if want_traj else None
        o = opts or default_opts()
        self._check(load_library().rs_simulate(self.ctx, B, _ptr(z), _ptr(v0), C.byref(ld), steps, float(dt),
                                               C.byref(o), _ptr(iters), _ptr(failed), _ptr(traj), _stream()),
                    "rs_simulate")
        return dict(z=z, iters=iters, failed=failed, traj=traj)

    def full_solve(self, u0, targets=None, force=None, opts: FullOpts | None = None, qbar=None, dt=0.0):
        """Full-space equilibria of B load cases from displacements u0 (B x nv x 3, float64,
        device); returns dict of device tensors (u, iters, status, relgrad, E)."""
        B = u0.shape[0]
        _dev(u0, torch.float64, (B, self.nv, 3), "u0")
        ld, _keep = self._load(B, targets, force, qbar, dt)
        u = u0.clone()
        dev = u0.device
        iters = torch.empty(B, dtype=torch.int32, device=dev)
        status = torch.empty(B, dtype=torch.int32, device=dev)
        relg = torch.empty(B, dtype=torch.float64, device=dev)
        E = torch.empty(B, dtype=torch.float64, device=dev)
        o = opts or default_full_opts()
        self._check(load_library().rs_full_solve(self.ctx, B, _ptr(u), C.byref(ld), C.byref(o), _ptr(iters),
                                                 _ptr(status), _ptr(relg), _ptr(E), _stream()), "rs_full_solve")
        return dict(u=u, iters=iters, status=status, relgrad=relg, E=E)

    def pca(self, store, r, iters=60):
        """(W (n x r), mean (n), evals (r), z_rest (r)) float64 device tensors: the
        mass-orthonormal PCA basis of the snapshot displacements `store` (N x n,
        context dtype, device) and the coordinates of the rest shape's projection."""
        _dev(store, self.tdtype, None, "store")
        if store.dim() != 2 or store.shape[1] != self.n:
            raise ValueError("store must be (N, 3 nv)")
        dev = store.device
        W = torch.empty((self.n, r), dtype=torch.float64, device=dev)
        mean = torch.empty(self.n, dtype=torch.float64, device=dev)
        ev = torch.empty(r, dtype=torch.float64, device=dev)
        zr = torch.empty(r, dtype=torch.float64, device=dev)
        self._check(load_library().rs_pca(self.ctx, store.shape[0], _ptr(store), r, iters, _ptr(W), _ptr(mean),
                                          _ptr(ev), _ptr(zr), _stream()), "rs_pca")
        return W, mean, ev, zr

    def lipschitz_loss(self, z1, z2, want_per_pair=True):
        B = z1.shape[0]
        _dev(z1, torch.float64, (B, self.r), "z1")
        _dev(z2, torch.float64, (B, self.r), "z2")
        dev = z1.device
        loss = torch.empty(1, dtype=torch.float64, device=dev)
        per = torch.empty(B, dtype=torch.float64, device=dev) if want_per_pair else None
        nval = torch.empty(1, dtype=torch.int32, device=dev)
        lmax = torch.empty(1, dtype=torch.float64, device=dev)
        self._check(load_library().rs_lipschitz_loss(self.ctx, B, _ptr(z1), _ptr(z2), _ptr(loss), _ptr(per),
                                                     _ptr(nval), _ptr(lmax), _stream()), "rs_lipschitz_loss")
        return dict(loss=loss, per_pair=per, n_valid=nval, lip_max=lmax)

    # -- kernel timing ------------------------------------------------------
    def kind_names(self):
        L = load_library()
        n = C.c_int32()
        self._check(L.rs_profile_get(self.ctx, -1, C.byref(n), None, 0, None, None, None, None), "rs_profile_get")
        name = C.create_string_buffer(64)
        out = []
        for i in range(n.value):
            self._check(L.rs_profile_get(self.ctx, i, C.byref(n), name, 64, None, None, None, None),
                        "rs_profile_get")
            out.append(name.value.decode())
        return out

    def profile(self, enable: bool, kinds=None):
        """Bracket launches with HIP events; `kinds` (names) limits which."""
        mask = 0
        if kinds:
            names = self.kind_names()
            for k in kinds:
                mask |= 1 << names.index(k)
        self._check(load_library().rs_profile(self.ctx, int(enable), mask), "rs_profile")

    def profile_read(self):
        L = load_library()
        n = C.c_int32()
        self._check(L.rs_profile_get(self.ctx, -1, C.byref(n), None, 0, None, None, None, None), "rs_profile_get")
        out = {}
        name = C.create_string_buffer(64)
        for i in range(n.value):
            la, ms, by, fl = C.c_int32(), C.c_double(), C.c_double(), C.c_double()
            self._check(L.rs_profile_get(self.ctx, i, C.byref(n), name, 64, C.byref(la), C.byref(ms), C.byref(by),
                                         C.byref(fl)), "rs_profile_get")
            if la.value:
                out[name.value.decode()] = dict(launches=la.value, ms=ms.value, bytes=by.value, flops=fl.value)
        return out


class Trainer:
    """The supervised autoencoder trainer of a context (rs_trainer_*): an ELU
    encoder (Ws, bs: host float64 arrays, W (out x in)) and the context's decoder,
    trained on a device store of snapshot displacements (N x 3 nv, context dtype)."""

    def __init__(self, ctx: Context, enc_Ws, enc_bs, dec_Ws, dec_bs, max_batch: int = 128):
        L = load_library()
        self.ctx = ctx
        keep = []
        Ws = [np.ascontiguousarray(W, dtype=np.float64) for W in enc_Ws]
        bs = [np.ascontiguousarray(b, dtype=np.float64) for b in enc_bs]
        keep.extend(Ws); keep.extend(bs)
        Wp = (_dp * len(Ws))(*[W.ctypes.data_as(_dp) for W in Ws])
        bp = (_dp * len(bs))(*[b.ctypes.data_as(_dp) for b in bs])
        keep.extend([Wp, bp])
        mlp = _Mlp(Ws[0].shape[1], len(Ws) - 1, Ws[0].shape[0] if len(Ws) > 1 else 0, Ws[-1].shape[0],
                   C.cast(Wp, C.POINTER(_dp)), C.cast(bp, C.POINTER(_dp)))
        dec = ctx._decoder_struct(dec_Ws, dec_bs, keep)
        t = C.c_void_p()
        ctx._check(L.rs_trainer_create(ctx.ctx, C.byref(mlp), C.byref(dec), max_batch, C.byref(t)),
                   "rs_trainer_create")
        self.t = t
        self.max_batch = max_batch
        self.enc_shapes = [(W.shape, b.shape) for W, b in zip(Ws, bs)]
        ne, nd = C.c_int64(), C.c_int64()
        ctx._check(L.rs_trainer_param_count(t, C.byref(ne), C.byref(nd)), "rs_trainer_param_count")
        self.n_enc, self.n_dec = ne.value, nd.value

    def close(self):
        if getattr(self, "t", None) is not None and _lib is not None:
            _lib.rs_trainer_destroy(self.t)
            self.t = None

    def __del__(self):
        self.close()

    def _store(self, store, idx, B):
        _dev(store, self.ctx.tdtype, None, "store")
        if store.dim() != 2 or store.shape[1] != self.ctx.n:
            raise ValueError("store must be (N, 3 nv)")
        if idx is not None:
            _dev(idx, torch.int32, None, "idx")
            B = idx.shape[0] if B is None else B
        elif B is None:
            B = store.shape[0]
        if idx is None and B > store.shape[0]:
            raise ValueError("B exceeds the store")
        return B

    def encode(self, store, idx=None, B=None):
        B = self._store(store, idx, B)
        z = torch.empty((B, self.ctx.r), dtype=torch.float64, device=store.device)
        self.ctx._check(load_library().rs_trainer_encode(self.t, B, _ptr(store), _ptr(idx), _ptr(z), _stream()),
                        "rs_trainer_encode")
        return z

    def grad(self, store, idx=None, B=None, lambda_ls=0.0, n_pairs=0, want_grads=False, losses=None):
        """Losses (2: L_C, L_LS) and, with want_grads, float64 gradients (encoder, decoder)."""
        B = self._store(store, idx, B)
        dev = store.device
        if losses is None:
            losses = torch.empty(2, dtype=torch.float64, device=dev)
        ge = torch.empty(self.n_enc, dtype=torch.float64, device=dev) if want_grads else None
        gd = torch.empty(self.n_dec, dtype=torch.float64, device=dev) if want_grads else None
        self.ctx._check(load_library().rs_trainer_grad(self.t, B, _ptr(store), _ptr(idx), float(lambda_ls),
                                                       int(n_pairs), _ptr(losses), _ptr(ge), _ptr(gd), _stream()),
                        "rs_trainer_grad")
        return losses, ge, gd

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.ctx._check(load_library().rs_trainer_adam(self.t, lr, beta1, beta2, eps, _stream()), "rs_trainer_adam")

    def params(self):
        """(encoder, decoder) packed parameters, context dtype, device."""
        dev = self.ctx.device
        e = torch.empty(self.n_enc, dtype=self.ctx.tdtype, device=dev)
        d = torch.empty(self.n_dec, dtype=self.ctx.tdtype, device=dev)
        self.ctx._check(load_library().rs_trainer_params(self.t, _ptr(e), _ptr(d), _stream()), "rs_trainer_params")
        return e, d

    def unpack_encoder(self, flat):
        out, off = [], 0
        for ws, bsh in self.enc_shapes:
            nw, nb = ws[0] * ws[1], bsh[0]
            out.append((flat[off:off + nw].reshape(ws), flat[off + nw:off + nw + nb]))
            off += nw + nb
        return out


class CubatureEnergy(torch.autograd.Function):
    """sum_b E(z_b; theta): the summed cubature energy (the potential loss of
    the unsupervised subspace construction, Sec. 3.2) as a differentiable
    function of the latent points z and of the packed decoder parameters
    theta.  Forward loads theta into the context and runs the library's
    reverse pass once; backward scales the saved gradients.  Usage:
    CubatureEnergy.apply(ctx, z, theta, targets, force, flags)."""

    @staticmethod
    def forward(fctx, rs_context, z, theta, targets=None, force=None, flags=0):
        rs_context.set_decoder_flat(theta)
        E, g, grad = rs_context.energy_param_grad(z.detach(), targets, force, flags)
        fctx.save_for_backward(g, grad)
        return E.sum()

    @staticmethod
    def backward(fctx, gout):
        g, grad = fctx.saved_tensors
        return None, gout * g, gout * grad, None, None, None
