"""MI355X-native preconditioned primal-dual TV/metal CT reconstruction.

Python binding of libctpd.so (include/ctpd.h).  Every step of the method runs
in the library's HIP kernels; this module only marshals arguments.  PyTorch
provides device memory (contiguous float32 CUDA/HIP tensors) and the current
stream.  There is no CPU fallback: without the built library, importing this
package raises ImportError, and a call on tensors that are not on the GPU
raises ValueError.

Method: C. Schiffer, "TV-regularized CT reconstruction and metal artifact
reduction using inequality constraints with preconditioning" (2018,
arXiv:1810.03275), Algorithm PDRQS1 (§4.4) with the inverse-norm
preconditioner (§4.3.1) and the normalization of §5.1.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Optional

import numpy as np
import torch

from . import _lib

_L = _lib.load()
# backprojector codes (CT_BP_*) to names, and the names' pixels per thread
_BP_NAMES = {v: k for k, v in _lib.BP_KERNELS.items() if v >= 0}
_BP_PIXELS = {"one_angle": 0, "pairs4": 4, "pairs8": 8}

__all__ = [
    "CtpdError", "Plan", "Precond", "Solver", "Launch", "radon_fwd", "radon_adj", "grad", "div",
    "prox_sino", "tv_project", "power_norm", "reconstruct", "pack_mask", "RadonFn",
    "RadonAdjFn", "estimate_d0", "lib",
]

lib = _L


class CtpdError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _L.ct_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.ERRORS.get(code, code)}: {msg}")
        self.code = code


def _check(code: int, where: str) -> None:
    if code != _lib.CT_OK:
        raise CtpdError(code, where)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, shape, name: str, dtype=torch.float32) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU (no CPU path exists)")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def pack_mask(mask) -> torch.Tensor:
    """Bool (N, M) metal-trace mask -> uint32 bitmask (N, ceil(M/32)) on the GPU
    (bit k & 31 of word k >> 5)."""
    m = mask.detach().cpu().numpy() if isinstance(mask, torch.Tensor) else np.asarray(mask)
    m = m.astype(bool)
    N, M = m.shape
    MW = (M + 31) // 32
    pad = np.zeros((N, MW * 32), dtype=bool)
    pad[:, :M] = m
    bits = np.packbits(pad, axis=1, bitorder="little").view(np.uint32)
    return torch.from_numpy(bits.astype(np.int32).copy()).cuda()


def _plan_opts(bp_kernel: str, fwd_angles_per_walk: int):
    if bp_kernel not in _lib.BP_KERNELS:
        raise ValueError(f"bp_kernel must be one of {sorted(_lib.BP_KERNELS)}")
    return _lib.CtPlanOpts(_lib.BP_KERNELS[bp_kernel], int(fwd_angles_per_walk))


def plan_check(n: int, n_angles: int, n_bins: int, h: float = 1.0, ds: float = 1.0,
               angles: Optional[np.ndarray] = None, bp_kernel: str = "auto",
               fwd_angles_per_walk: int = 0) -> int:
    """Host-only replay of the forward projector's walk over the plan that
    Plan(...) would build; returns the number of (strip, row) steps checked and
    raises CtpdError if a staged window or a skipped row is wrong."""
    g = _lib.CtGeom(n, n_angles, n_bins, h, ds)
    steps = ctypes.c_int64(0)
    ptr = None
    if angles is not None:
        a = np.ascontiguousarray(angles, dtype=np.float64)
        if a.shape != (n_angles,):
            raise ValueError("angles must have shape (n_angles,)")
        ptr = a.ctypes.data_as(ctypes.c_void_p)
    opts = _plan_opts(bp_kernel, fwd_angles_per_walk)
    _check(_L.ct_plan_check_ex(ctypes.byref(g), ptr, ctypes.byref(opts), ctypes.byref(steps)),
           "ct_plan_check")
    return int(steps.value)


class Plan:
    """Projector plan for an n x n image, N angles, M bins (§3.1).

    bp_kernel: backprojector of standalone calls and untuned solvers ("auto",
    "one_angle", "pairs4", "pairs8"); fwd_angles_per_walk: angles sharing one
    walk of R_h (0 automatic, 1, 2 or 4; a mode whose windows do not fit falls
    back to the next)."""

    def __init__(self, n: int, n_angles: int, n_bins: int, h: float = 1.0, ds: float = 1.0,
                 angles: Optional[np.ndarray] = None, bp_kernel: str = "auto",
                 fwd_angles_per_walk: int = 0):
        self.n, self.n_angles, self.n_bins, self.h, self.ds = n, n_angles, n_bins, h, ds
        g = _lib.CtGeom(n, n_angles, n_bins, h, ds)
        handle = ctypes.c_void_p()
        opts = _plan_opts(bp_kernel, fwd_angles_per_walk)
        ptr = None
        if angles is not None:
            a = np.ascontiguousarray(angles, dtype=np.float64)
            if a.shape != (n_angles,):
                raise ValueError("angles must have shape (n_angles,)")
            ptr = a.ctypes.data_as(ctypes.c_void_p)
        _check(_L.ct_plan_create_ex(ctypes.byref(g), ptr, ctypes.byref(opts),
                                    ctypes.byref(handle)), "ct_plan_create")
        self._h = handle

    @property
    def handle(self):
        return self._h

    def layout(self) -> dict:
        """The plan's forward-projector layout (angles per walk, groups,
        workgroups per problem) and default backprojector (its name, and
        mirror-pair pixels per thread, 0: one angle at a time)."""
        o = (ctypes.c_int32 * 4)()
        _check(_L.ct_plan_layout(self.handle, o), "ct_plan_layout")
        name = _BP_NAMES[o[3]]
        return {"angles_per_walk": o[0], "fwd_groups": o[1], "fwd_workgroups": o[2],
                "bp_kernel": name, "bp_pair_pixels": _BP_PIXELS[name]}

    def close(self):
        if self._h:
            _L.ct_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def radon_fwd(self, img: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        p = _dev(img, (self.n, self.n), "img")
        if out is None:
            out = torch.empty((self.n_angles, self.n_bins), device=img.device, dtype=torch.float32)
        q = _dev(out, (self.n_angles, self.n_bins), "out")
        _check(_L.ct_radon_fwd(self._h, p, q, _stream()), "ct_radon_fwd")
        return out

    def radon_adj(self, sino: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        p = _dev(sino, (self.n_angles, self.n_bins), "sino")
        if out is None:
            out = torch.empty((self.n, self.n), device=sino.device, dtype=torch.float32)
        q = _dev(out, (self.n, self.n), "out")
        _check(_L.ct_radon_adj(self._h, p, q, _stream()), "ct_radon_adj")
        return out


def radon_fwd(plan: Plan, img: torch.Tensor, out=None) -> torch.Tensor:
    """sino = R_h img (§3.1)."""
    return plan.radon_fwd(img, out)


def radon_adj(plan: Plan, sino: torch.Tensor, out=None) -> torch.Tensor:
    """img = R_h^* sino (§3.1)."""
    return plan.radon_adj(sino, out)


def estimate_d0(plan: Plan, u_rec: torch.Tensor, threshold: float, radius: int = 5,
                kappa: float = 1e-3, u0: Optional[torch.Tensor] = None, c0: float = 0.8):
    """Metal trace from a reconstruction (results chapter, real metal
    artifacts): pixels of u_rec above threshold, dilated by a disk of the given
    radius (pixels), projected; D0 = {R_h chi > kappa}.  Returns
    (chi [n][n], R_h chi [N][M], packed D0 mask [N][ceil(M/32)] int32, bound),
    bound = c0 u0 on D0 (0 elsewhere) when u0 is given, else None."""
    n, N, M = plan.n, plan.n_angles, plan.n_bins
    dev = u_rec.device
    chi = torch.empty((n, n), device=dev, dtype=torch.float32)
    proj = torch.empty((N, M), device=dev, dtype=torch.float32)
    mask = torch.empty((N, (M + 31) // 32), device=dev, dtype=torch.int32)
    bound = None
    u0p = None
    if u0 is not None:
        u0p = _dev(u0, (N, M), "u0")
        bound = torch.empty((N, M), device=dev, dtype=torch.float32)
    _check(_L.ct_d0_estimate(plan.handle, _dev(u_rec, (n, n), "u_rec"), float(threshold),
                             int(radius), float(kappa), chi.data_ptr(), proj.data_ptr(),
                             mask.data_ptr(), u0p, float(c0),
                             bound.data_ptr() if bound is not None else None, _stream()),
           "ct_d0_estimate")
    return chi, proj, mask, bound


def grad(u: torch.Tensor, h: float = 1.0, out=None) -> torch.Tensor:
    """Forward-difference gradient, planar (2, n, n) (§3.1)."""
    n = u.shape[0]
    p = _dev(u, (n, n), "u")
    if out is None:
        out = torch.empty((2, n, n), device=u.device, dtype=torch.float32)
    _check(_L.ct_grad(n, h, p, _dev(out, (2, n, n), "out"), _stream()), "ct_grad")
    return out


def div(pf: torch.Tensor, h: float = 1.0, out=None) -> torch.Tensor:
    """div_h = -nabla_h^T (§3.1)."""
    n = pf.shape[1]
    p = _dev(pf, (2, n, n), "p")
    if out is None:
        out = torch.empty((n, n), device=pf.device, dtype=torch.float32)
    _check(_L.ct_div(n, h, p, _dev(out, (n, n), "out"), _stream()), "ct_div")
    return out


def prox_sino(q: torch.Tensor, step: float, u0: torch.Tensor, bound: Optional[torch.Tensor],
              mask_bits: Optional[torch.Tensor], out=None) -> torch.Tensor:
    """Sinogram resolvent of §3.3/§4.4 (mask_bits from pack_mask, or None)."""
    N, M = q.shape
    if out is None:
        out = torch.empty_like(q)
    mb = _dev(mask_bits, (N, (M + 31) // 32), "mask", torch.int32) if mask_bits is not None else None
    bd = _dev(bound, (N, M), "bound") if bound is not None else None
    _check(_L.ct_prox_sino(N, M, _dev(q, (N, M), "q"), step, _dev(u0, (N, M), "u0"), bd, mb,
                           _dev(out, (N, M), "out"), _stream()), "ct_prox_sino")
    return out


def tv_project(q: torch.Tensor, radius: float, out=None) -> torch.Tensor:
    """Pointwise projection onto the Euclidean ball (§3.3)."""
    n = q.shape[1]
    if out is None:
        out = torch.empty_like(q)
    _check(_L.ct_tv_project(n, _dev(q, (2, n, n), "q"), radius, _dev(out, (2, n, n), "out"),
                            _stream()), "ct_tv_project")
    return out


class Precond:
    """M^{-1} of §4.4: F^{-1}( F(y) rho / (sigma^2 c + (sigma tau)^2 lambda_Delta rho) )."""

    def __init__(self, n: int, sigma: float, tau: float, c: float, eps: float):
        self.n = n
        h = ctypes.c_void_p()
        _check(_L.ct_precond_create(n, sigma, tau, c, eps, ctypes.byref(h)), "ct_precond_create")
        self._h = h

    def apply(self, y: torch.Tensor, out=None) -> torch.Tensor:
        if out is None:
            out = torch.empty_like(y)
        _check(_L.ct_precond_apply(self._h, _dev(y, (self.n, self.n), "y"),
                                   _dev(out, (self.n, self.n), "out"), _stream()),
               "ct_precond_apply")
        return out

    def __del__(self):
        try:
            if self._h:
                _L.ct_precond_destroy(self._h)
                self._h = ctypes.c_void_p()
        except Exception:
            pass


def power_norm(plan: Plan, iters: int = 30, x0: Optional[torch.Tensor] = None) -> float:
    """sqrt(lambda_max(R^* R)) by power iteration (§5.1); synchronizes."""
    out = ctypes.c_double()
    xp = _dev(x0, (plan.n, plan.n), "x0") if x0 is not None else None
    _check(_L.ct_power_norm(plan.handle, iters, xp, ctypes.byref(out), _stream()),
           "ct_power_norm")
    return out.value


@dataclasses.dataclass
class Launch:
    """Launch choices of a solver's iteration (ct_params fields).  None: chosen
    by the set-up tuning.  bp_slices: angle slices of R_h^* (1..16);
    bp_kernel: "one_angle", "pairs4" or "pairs8"; tv_blocks: workgroups of
    the gradient-side update inside R_h's launch; tune=False: the plan's
    defaults instead of timing; defer / fuse_tv / graph=False: the slice sum,
    the gradient-side update or the iterations as launches of their own
    (same arithmetic); tune_cache: path of a JSON file of tuning results;
    fwd_walk: angles per walk of R_h in the iteration (1, 2 or 4; None: the
    plan's when its walk was fixed, else tuned)."""
    bp_slices: Optional[int] = None
    bp_kernel: Optional[str] = None
    tv_blocks: Optional[int] = None
    fwd_walk: Optional[int] = None
    tune: bool = True
    defer: bool = True
    fuse_tv: bool = True
    graph: bool = True
    tune_cache: Optional[str] = None

    def fill(self, p) -> None:
        p.bp_slices = int(self.bp_slices or 0)
        if self.bp_kernel is not None and self.bp_kernel not in _lib.BP_KERNELS:
            raise ValueError(f"bp_kernel must be one of {sorted(_lib.BP_KERNELS)}")
        p.bp_kernel = _lib.BP_KERNELS[self.bp_kernel or "auto"]
        p.tv_blocks = int(self.tv_blocks or 0)
        p.options = ((0 if self.tune else _lib.CT_OPT_NO_TUNE)
                     | (0 if self.defer else _lib.CT_OPT_NO_DEFER)
                     | (0 if self.fuse_tv else _lib.CT_OPT_SEPARATE_TV)
                     | (0 if self.graph else _lib.CT_OPT_NO_GRAPH))
        p.tune_cache = self.tune_cache.encode() if self.tune_cache else None
        p.fwd_walk = int(self.fwd_walk or 0)


def power_norm_noalloc(plan: Plan, iters: int = 30, x0: Optional[torch.Tensor] = None) -> float:
    """power_norm without any device allocation (scratch in the library's
    static device array; see ct_power_norm_noalloc); synchronizes."""
    out = ctypes.c_double()
    xp = _dev(x0, (plan.n, plan.n), "x0") if x0 is not None else None
    _check(_L.ct_power_norm_noalloc(plan.handle, iters, xp, ctypes.byref(out), _stream()),
           "ct_power_norm_noalloc")
    return out.value


VALU_PROBE_KINDS = {"fma_f32": (0, 1), "add_f32": (1, 1), "xad_u32": (2, 1),
                    "xad_u32+cvt_f32_u32": (3, 2), "add_u64": (4, 1)}
# name -> (kind, instructions per chain and round)


def valu_probe(blocks: int, iters: int, out: torch.Tensor, kind: str = "fma_f32") -> int:
    """Launch the vector issue-rate probe (ct_valu_probe) on the current
    stream and return its wave-instruction count, blocks * 4 * iters * 16 * I
    (kinds and I in VALU_PROBE_KINDS).  out: float32 device tensor of at least
    `blocks` elements (it only keeps the work live)."""
    if out.dtype != torch.float32 or not out.is_cuda or out.numel() < blocks:
        raise ValueError("out must be a float32 device tensor of at least `blocks` elements")
    k, per = VALU_PROBE_KINDS[kind]
    _check(_L.ct_valu_probe(blocks, iters, k, out.data_ptr(), _stream()), "ct_valu_probe")
    return blocks * 4 * iters * 16 * per


def copy_probe(src: torch.Tensor, dst: torch.Tensor, blocks: int) -> None:
    """Launch the streaming copy probe (ct_copy_probe) of src into dst (device
    tensors of equal byte size) on the current stream."""
    nbytes = src.numel() * src.element_size()
    if (not src.is_cuda or not dst.is_cuda or not src.is_contiguous() or not dst.is_contiguous()
            or dst.numel() * dst.element_size() != nbytes):
        raise ValueError("src and dst must be contiguous device tensors of the same byte size")
    _check(_L.ct_copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, blocks, _stream()),
           "ct_copy_probe")


def _params(sigma, tau, eps, c, c_safety, beta, k_max, gap_every, power_iters, validate,
            start_norm, start_precond, n, nonneg=False, method="pdrqs1", precond="invnorm",
            launch=None):
    p = _lib.CtParams()
    _L.ct_params_default(ctypes.byref(p))
    if launch is not None:
        (Launch(**launch) if isinstance(launch, dict) else launch).fill(p)
    p.sigma, p.tau, p.eps = sigma, tau, eps
    p.c = c if c is not None else 0.0
    p.c_safety = c_safety
    p.beta = beta if beta is not None else 0.0
    p.k_max, p.gap_every, p.power_iters = k_max, gap_every, power_iters
    if method not in _lib.METHODS:
        raise ValueError(f"method must be one of {sorted(_lib.METHODS)}")
    if precond not in _lib.PRECONDS:
        raise ValueError(f"precond must be one of {sorted(_lib.PRECONDS)}")
    p.flags = ((_lib.CT_FLAG_VALIDATE if validate else 0)
               | (_lib.CT_FLAG_NONNEG if nonneg else 0)
               | (_lib.METHODS[method] << _lib.CT_METHOD_SHIFT)
               | (_lib.PRECONDS[precond] << _lib.CT_PRECOND_SHIFT))
    p.start_norm = _dev(start_norm, (n, n), "start_norm") if start_norm is not None else None
    p.start_precond = (_dev(start_precond, (n, n), "start_precond")
                       if start_precond is not None else None)
    return p


def _problem(plan: Plan, sino, mask_bits, bound, lam, bound_scalar=0.0):
    N, M = plan.n_angles, plan.n_bins
    pr = _lib.CtProblem()
    pr.sino = _dev(sino, (N, M), "sino")
    pr.mask = _dev(mask_bits, (N, (M + 31) // 32), "mask", torch.int32) if mask_bits is not None else None
    pr.bound = _dev(bound, (N, M), "bound") if bound is not None else None
    pr.bound_scalar = bound_scalar
    pr.lambda_ = lam
    return pr


class Solver:
    """PDRQS1 solver state on the GPU (§4.4).  Keeps references to its inputs."""

    def __init__(self, plan: Plan, sino: torch.Tensor, lam: float,
                 mask_bits: Optional[torch.Tensor] = None, bound: Optional[torch.Tensor] = None,
                 *, sigma: float = 1.0, tau: float = 1.0 / math.sqrt(8.0), eps: float = 0.3,
                 c: Optional[float] = None, c_safety: float = 1.1, beta: Optional[float] = None,
                 power_iters: int = 30, validate: bool = False,
                 start_norm: Optional[torch.Tensor] = None,
                 start_precond: Optional[torch.Tensor] = None, bound_scalar: float = 0.0,
                 nonneg: bool = False, method: str = "pdrqs1", cg_steps: int = 1,
                 mu: float = 1.0, precond: str = "invnorm", launch=None):
        self.plan = plan
        self._keep = (sino, mask_bits, bound, start_norm, start_precond)
        prob = _problem(plan, sino, mask_bits, bound, lam, bound_scalar)
        prm = _params(sigma, tau, eps, c, c_safety, beta, 0, 0, power_iters, validate,
                      start_norm, start_precond, plan.n, nonneg, method, precond, launch)
        h = ctypes.c_void_p()
        _check(_L.ct_solver_create(plan.handle, ctypes.byref(prob), ctypes.byref(prm), _stream(),
                                   ctypes.byref(h)), "ct_solver_create")
        self._h = h
        if method == "admm":
            # ADMM (§4.6): PCG steps per iteration and the augmented-Lagrangian weight
            _check(_L.ct_solver_set_admm(h, int(cg_steps), float(mu)), "ct_solver_set_admm")

    def info(self) -> dict:
        o = (ctypes.c_double * 4)()
        _check(_L.ct_solver_info(self._h, o), "ct_solver_info")
        return {"beta": o[0], "c": o[1], "lam_t": o[2], "iters": int(o[3])}

    def set_fit(self, fit: str, aux: Optional[torch.Tensor] = None) -> None:
        """Data-term variant (§3.5): standard, weighted (aux = weights),
        ignore, everywhere (aux = u0 on every bin), hard.  Before the first
        iteration."""
        if fit not in _lib.FITS:
            raise ValueError(f"fit must be one of {sorted(_lib.FITS)}")
        N, M = self.plan.n_angles, self.plan.n_bins
        ptr = _dev(aux, self._lead() + (N, M), "aux") if aux is not None else None
        self._keep_aux = aux
        _check(_L.ct_solver_set_fit(self._h, _lib.FITS[fit], ptr, _stream()),
               "ct_solver_set_fit")

    def step(self, k: int = 1) -> None:
        _check(_L.ct_pd_step(self._h, k, _stream()), "ct_pd_step")

    def step_timed(self, k: int) -> dict:
        """k iterations launched one by one; average ms per iteration of each phase."""
        o = (ctypes.c_double * 5)()
        _check(_L.ct_pd_step_timed(self._h, k, o, _stream()), "ct_pd_step_timed")
        return dict(zip(("radon_adj", "precond", "radon_fwd", "tv_update", "total"), list(o)))

    nb = 1

    def _lead(self):
        return () if self.nb == 1 else (self.nb,)

    def layout(self) -> dict:
        o = (ctypes.c_int32 * 6)()
        _check(_L.ct_solver_layout(self._h, o), "ct_solver_layout")
        name = "one_angle" if o[4] == 1 else f"pairs{o[5]}"
        return {"problems": o[0], "bp_slices": o[1], "angles_per_walk": o[2], "fwd_groups": o[3],
                "bp_angles_per_position": o[4], "bp_pair_pixels": o[5], "bp_kernel": name}

    def tuning(self) -> dict:
        """How the launch choices were made: source (fixed, timed, plan,
        file), candidates timed, gradient-side workgroups in R_h's launch (0:
        own launch), whether the tune cache file was written."""
        o = (ctypes.c_int32 * 4)()
        _check(_L.ct_solver_tuning(self._h, o), "ct_solver_tuning")
        return {"source": ("fixed", "timed", "plan", "file")[o[0]], "timed": o[1],
                "tv_blocks": o[2], "saved": bool(o[3])}

    def export(self):
        n, N, M = self.plan.n, self.plan.n_angles, self.plan.n_bins
        dev = torch.device("cuda")
        L = self._lead()
        u = torch.empty(L + (n, n), device=dev)
        vb1 = torch.empty(L + (N, M), device=dev)
        vb2 = torch.empty(L + (2, n, n), device=dev)
        _check(_L.ct_state_export(self._h, u.data_ptr(), vb1.data_ptr(), vb2.data_ptr(),
                                  _stream()), "ct_state_export")
        return u, vb1, vb2

    def import_state(self, u, vb1, vb2) -> None:
        n, N, M = self.plan.n, self.plan.n_angles, self.plan.n_bins
        L = self._lead()
        _check(_L.ct_state_import(self._h, _dev(u, L + (n, n), "u"),
                                  _dev(vb1, L + (N, M), "vb1"),
                                  _dev(vb2, L + (2, n, n), "vb2"), _stream()), "ct_state_import")

    def export_ubar(self) -> torch.Tensor:
        """bar u of the u >= 0 variant."""
        n = self.plan.n
        ub = torch.empty(self._lead() + (n, n), device=torch.device("cuda"))
        _check(_L.ct_state_export_ubar(self._h, ub.data_ptr(), _stream()),
               "ct_state_export_ubar")
        return ub

    def import_ubar(self, ub) -> None:
        n = self.plan.n
        _check(_L.ct_state_import_ubar(self._h, _dev(ub, self._lead() + (n, n), "ubar"),
                                       _stream()), "ct_state_import_ubar")

    def gap(self) -> np.ndarray:
        """FP64 record (6 values; (nb, 6) for a batch)."""
        o = (ctypes.c_double * (6 * self.nb))()
        _check(_L.ct_gap(self._h, o, _stream()), "ct_gap")
        r = np.array(list(o), dtype=np.float64)
        return r if self.nb == 1 else r.reshape(self.nb, 6)

    def close(self):
        if self._h:
            _L.ct_solver_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SolverBatch(Solver):
    """nb problems of one geometry advanced together (one launch per kernel
    for all of them); state tensors carry a leading batch dimension."""

    def __init__(self, plan: Plan, sinos, lam: float, masks=None, bounds=None, *,
                 sigma: float = 1.0, tau: float = 1.0 / math.sqrt(8.0), eps: float = 0.3,
                 c: Optional[float] = None, c_safety: float = 1.1, beta: Optional[float] = None,
                 power_iters: int = 30, validate: bool = False,
                 start_norm: Optional[torch.Tensor] = None,
                 start_precond: Optional[torch.Tensor] = None, bound_scalars=None,
                 nonneg: bool = False, launch=None):
        self.plan = plan
        nb = len(sinos)
        masks = masks if masks is not None else [None] * nb
        bounds = bounds if bounds is not None else [None] * nb
        bsc = bound_scalars if bound_scalars is not None else [0.0] * nb
        if not (len(masks) == len(bounds) == len(bsc) == nb) or nb < 1:
            raise ValueError("sinos, masks, bounds and bound_scalars need one entry per problem")
        self.nb = nb
        self._keep = (list(sinos), list(masks), list(bounds), start_norm, start_precond)
        probs = (_lib.CtProblem * nb)()
        for b in range(nb):
            probs[b] = _problem(plan, sinos[b], masks[b], bounds[b], lam, bsc[b])
        prm = _params(sigma, tau, eps, c, c_safety, beta, 0, 0, power_iters, validate,
                      start_norm, start_precond, plan.n, nonneg, launch=launch)
        h = ctypes.c_void_p()
        _check(_L.ct_solver_create_batch(plan.handle, probs, nb, ctypes.byref(prm), _stream(),
                                         ctypes.byref(h)), "ct_solver_create_batch")
        self._h = h


class SolverGroup:
    """Solvers (any geometries, same iteration count) stepped together from one
    HIP graph.  Keeps references to the solvers; close() before they go."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s._h.value for s in self.solvers])
        h = ctypes.c_void_p()
        _check(_L.ct_group_create(arr, len(self.solvers), ctypes.byref(h)), "ct_group_create")
        self._h = h

    def step(self, k: int = 1) -> None:
        _check(_L.ct_group_step(self._h, k, _stream()), "ct_group_step")

    def close(self):
        if self._h:
            _L.ct_group_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reconstruct_batched(problems, *, k_max: int = 100, gap_every: int = 0, sigma: float = 1.0,
                        tau: float = 1.0 / math.sqrt(8.0), eps: float = 0.3,
                        c: Optional[float] = None, c_safety: float = 1.1,
                        beta: Optional[float] = None, power_iters: int = 30,
                        validate: bool = False, nonneg: bool = False, launch=None):
    """PDRQS1 solves of many problems, any mix of geometries.  problems: list of
    dicts with keys plan, sino, lam and optionally mask_bits, bound,
    bound_scalar.  Problems sharing a plan and lambda run as one batch; all
    batches' iterations replay as one HIP graph.  beta and c (if not given)
    are estimated per batch.  Returns ([u_i], report (count, records, 6) or
    None)."""
    count = len(problems)
    if count < 1:
        raise ValueError("no problems")
    plans = (ctypes.c_void_p * count)()
    probs = (_lib.CtProblem * count)()
    outs = (ctypes.c_void_p * count)()
    us = []
    for i, pr in enumerate(problems):
        plan = pr["plan"]
        plans[i] = plan.handle.value
        probs[i] = _problem(plan, pr["sino"], pr.get("mask_bits"), pr.get("bound"), pr["lam"],
                            pr.get("bound_scalar", 0.0))
        u = torch.empty((plan.n, plan.n), device=pr["sino"].device, dtype=torch.float32)
        us.append(u)
        outs[i] = u.data_ptr()
    prm = _params(sigma, tau, eps, c, c_safety, beta, k_max, gap_every, power_iters, validate,
                  None, None, problems[0]["plan"].n, nonneg, launch=launch)
    nrec = k_max // gap_every if gap_every > 0 else 0
    rep = (ctypes.c_double * max(1, 6 * nrec * count))()
    _check(_L.ct_reconstruct_batched(count, plans, probs, ctypes.byref(prm), outs,
                                     rep if nrec else None, 6 * nrec * count, _stream()),
           "ct_reconstruct_batched")
    report = (np.array(list(rep), dtype=np.float64).reshape(count, nrec, 6) if nrec else None)
    return us, report


def objective(plan: Plan, sino: torch.Tensor, lam: float, u: torch.Tensor, mask_bits=None,
              bound=None, bound_scalar: float = 0.0) -> np.ndarray:
    """(1/2 fit off D0, lambda TV, constraint violation) of (C_h) at u, FP64."""
    prob = _problem(plan, sino, mask_bits, bound, lam, bound_scalar)
    o = (ctypes.c_double * 3)()
    _check(_L.ct_objective(plan.handle, ctypes.byref(prob), _dev(u, (plan.n, plan.n), "u"), o,
                           _stream()), "ct_objective")
    return np.array(list(o), dtype=np.float64)


def reconstruct(plan: Plan, sino: torch.Tensor, lam: float, mask_bits=None, bound=None, *,
                k_max: int = 100, gap_every: int = 0, sigma: float = 1.0,
                tau: float = 1.0 / math.sqrt(8.0), eps: float = 0.3, c: Optional[float] = None,
                c_safety: float = 1.1, beta: Optional[float] = None, power_iters: int = 30,
                validate: bool = False, start_norm=None, start_precond=None,
                bound_scalar: float = 0.0, nonneg: bool = False, method: str = "pdrqs1",
                launch=None):
    """One-shot solve (PDRQS1 by default; nonneg: with u >= 0, §4.5); returns
    (u, report (records x 6) or None)."""
    prob = _problem(plan, sino, mask_bits, bound, lam, bound_scalar)
    prm = _params(sigma, tau, eps, c, c_safety, beta, k_max, gap_every, power_iters, validate,
                  start_norm, start_precond, plan.n, nonneg, method, launch=launch)
    u = torch.empty((plan.n, plan.n), device=sino.device, dtype=torch.float32)
    nrec = k_max // gap_every if gap_every > 0 else 0
    rep = (ctypes.c_double * max(1, 6 * nrec))()
    _check(_L.ct_reconstruct(plan.handle, ctypes.byref(prob), ctypes.byref(prm), u.data_ptr(),
                             rep if nrec else None, 6 * nrec, _stream()), "ct_reconstruct")
    report = np.array(list(rep), dtype=np.float64).reshape(-1, 6)[:nrec] if nrec else None
    return u, report


class Tape:
    """K unrolled PDRQS1 iterations of a solver (from the zero state), kept for
    the reverse sweep (checkpoints every `every` iterations)."""

    def __init__(self, solver: Solver, K: int, every: int = 10):
        self.solver = solver
        h = ctypes.c_void_p()
        _check(_L.ct_unrolled_forward(solver._h, K, every, ctypes.byref(h), _stream()),
               "ct_unrolled_forward")
        self._h = h
        self.K = K

    def backward(self, gbar: torch.Tensor):
        """dL/du0 (solver's sinogram layout) and dL/dlambda per problem."""
        sv = self.solver
        n, N, M = sv.plan.n, sv.plan.n_angles, sv.plan.n_bins
        L = sv._lead()
        g = gbar.detach().to(torch.float32).contiguous()
        ptr = _dev(g, L + (n, n), "gbar")
        du0 = torch.empty(L + (N, M), device=g.device, dtype=torch.float32)
        dl = (ctypes.c_double * sv.nb)()
        _check(_L.ct_unrolled_backward(self._h, ptr, du0.data_ptr(), dl, _stream()),
               "ct_unrolled_backward")
        return du0, np.array(list(dl), dtype=np.float64)

    def close(self):
        if self._h:
            _L.ct_tape_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class UnrolledPD(torch.autograd.Function):
    """u_K of K unrolled PDRQS1 iterations (§4.4) from the zero state, as a
    differentiable function of the data u0 (nb, N, M) and of lambda (a 0-d
    tensor).  The backward pass is the reverse sweep of the iteration with
    checkpoints every `every` iterations (beta and c held fixed: they depend
    on the geometry only).  Returns (nb, n, n)."""

    @staticmethod
    def forward(ctx, sinos, lam, plan, masks, bounds, K, every, opts):
        nb = sinos.shape[0]
        sv = SolverBatch(plan, [sinos[b].detach() for b in range(nb)], float(lam), masks,
                         bounds, **(opts or {}))
        tape = Tape(sv, K, every)
        u = sv.export()[0]
        ctx.tape = tape
        return u.reshape(nb, plan.n, plan.n)

    @staticmethod
    def backward(ctx, gu):
        tape = ctx.tape
        nb = tape.solver.nb
        sv = tape.solver
        g = gu.reshape(sv._lead() + (sv.plan.n, sv.plan.n))
        du0, dl = tape.backward(g)
        dlam = torch.tensor(float(dl.sum()), dtype=torch.float32, device=gu.device)
        return (du0.reshape(nb, sv.plan.n_angles, sv.plan.n_bins), dlam, None, None, None, None,
                None, None)


def unrolled_pd(plan: Plan, sinos: torch.Tensor, lam: torch.Tensor, masks=None, bounds=None,
                K: int = 50, every: int = 10, **opts) -> torch.Tensor:
    """Differentiable u_K for the batch of sinograms sinos (nb, N, M)."""
    return UnrolledPD.apply(sinos, lam, plan, masks, bounds, K, every, opts)


class RadonFn(torch.autograd.Function):
    """sino = R_h img; the backward pass is R_h^* (the exact transpose, §3.1)."""

    @staticmethod
    def forward(ctx, img, plan):
        ctx.plan = plan
        return plan.radon_fwd(img.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.radon_adj(g.contiguous()), None


class RadonAdjFn(torch.autograd.Function):
    """img = R_h^* sino; the backward pass is R_h."""

    @staticmethod
    def forward(ctx, sino, plan):
        ctx.plan = plan
        return plan.radon_adj(sino.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.radon_fwd(g.contiguous()), None
