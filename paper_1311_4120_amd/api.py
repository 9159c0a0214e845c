"""Torch-facing wrapper over the C ABI.  PyTorch supplies device memory and
the stream; every computation is a kernel of libjgb.so."""
from __future__ import annotations

import ctypes
import math
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import check, lib

_KERNELS = {"coulomb3d": _lib.COULOMB_3D, "coulomb2d": _lib.COULOMB_2D, "dipole3d": _lib.DIPOLE_3D,
            "dipole2d": _lib.DIPOLE_2D, "poisson2d": _lib.POISSON_2D}
_RULES = {"theta": _lib.THETA_GL, "costheta": _lib.COSTHETA_GL}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


# the plan flags a Batch member or a GPE driver may set by keyword
_FLAG_KWARGS = ("interp_tiles", "spread_rings", "radial_ggq", "gaussian_kernel")


def _make_params(n, box, kernel, nodes, eps, precision, lam, axis, theta_rule, kmax, device, stream,
                 autotune=False, split=False, window=(0.0, 0.0), axis2=None, alpha=0.0, interp_tiles=False,
                 spread_rings=False, radial_ggq=False, gaussian_kernel=False):
    dim = len(n)
    kern = _KERNELS.get(kernel, kernel)
    rule = _RULES.get(theta_rule, theta_rule)
    dev = torch.cuda.current_device() if device is None else int(device)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    p = _lib.Params()
    p.struct_size = ctypes.sizeof(_lib.Params)
    p.dim = dim
    for i in range(dim):
        p.n[i] = int(n[i])
        p.box[i] = float(box[i])
    p.kernel = int(kern)
    for i in range(3):
        p.dipole_axis[i] = float(axis[i]) if i < len(axis) else 0.0
    p.lam = float(lam)
    p.eps = float(eps)
    p.precision = _lib.FP64 if precision == "fp64" else _lib.MIXED
    if dim == 3:
        p.n_r, p.n_theta, p.n_phi = (int(v) for v in nodes)
    else:
        p.n_r, p.n_phi = int(nodes[0]), int(nodes[-1])
        p.n_theta = 1
    p.theta_rule = int(rule)
    p.kmax = float(kmax)
    p.device = dev
    p.stream = ctypes.c_void_p(st.cuda_stream)
    p.flags = ((_lib.FLAG_AUTOTUNE if autotune else 0) | (_lib.FLAG_SPLIT if split else 0)
               | (_lib.FLAG_INTERP_TILES if interp_tiles else 0) | (_lib.FLAG_SPREAD_RINGS if spread_rings else 0)
               | (_lib.FLAG_RADIAL_GGQ if radial_ggq else 0) | (_lib.FLAG_GAUSSIAN_KERNEL if gaussian_kernel else 0))
    for i in range(2):
        p.window[i] = float(window[i]) if i < len(window) else 0.0
    for i in range(3):
        p.dipole_axis2[i] = float(axis2[i]) if axis2 is not None and i < len(axis2) else 0.0
    p.alpha = float(alpha)
    return p, dev, st


class Plan:
    """A planned free-space convolution u = U*rho on one uniform grid.

    n, box:    grid points N_j and full side lengths R_j (2 or 3 axes)
    kernel:    "coulomb3d", "coulomb2d", "dipole3d", "dipole2d" or "poisson2d" (or the jgb_kernel ints)
    axis:      dipole orientation n (a unit 3-vector, also for "dipole2d")
    axis2:     second orientation m (None: m = n)
    alpha:     the 2.5D dipole's constant
    nodes:     (n_r, n_theta, n_phi) for 3D, (n_r, n_phi) for 2D
    precision: "fp64" or "mixed"
    split:     evaluate by Algorithm 2 (window p, I1 on the regular grid, I2 on
               the nodes); then kmax is I2's cut-off and window the scales
               (3D: (a, 0); 2D: (R0, R1); zeros: the defaults)
    interp_tiles: interpolate by tiles on the matrix cores (3D)
    spread_rings: spread ring by ring, each ring's nodes summed over the first
               two axes on the matrix cores and the ring sums spread along
               the last (3D)
    radial_ggq: radial nodes by the generalized Gaussian rule for band-limited
               integrands (prolate spheroidal) instead of Gauss-Legendre
    gaussian_kernel: spread and interpolate with the paper's Gaussian (12
               points per axis, about six digits; eps >= 1e-6) instead of the
               exponential of a semicircle
    """

    def __init__(self, n: Sequence[int], box: Sequence[float], kernel, nodes: Sequence[int],
                 eps: float = 1e-10, precision: str = "fp64", lam: float = 1.0,
                 axis: Sequence[float] = (0.0, 0.0, 1.0), theta_rule="theta", kmax: float = 0.0,
                 device: Optional[int] = None, stream: Optional[torch.cuda.Stream] = None, autotune: bool = False,
                 split: bool = False, window: Sequence[float] = (0.0, 0.0),
                 axis2: Optional[Sequence[float]] = None, alpha: float = 0.0, interp_tiles: bool = False,
                 spread_rings: bool = False, radial_ggq: bool = False, gaussian_kernel: bool = False):
        p, dev, st = _make_params(n, box, kernel, nodes, eps, precision, lam, axis, theta_rule, kmax, device, stream,
                                  autotune, split, window, axis2, alpha, interp_tiles, spread_rings, radial_ggq,
                                  gaussian_kernel)
        self._init_from(p, dev, st, box)
        h = ctypes.c_void_p()
        check(lib.jgb_plan(ctypes.byref(p), ctypes.byref(h)))
        self._set_handle(h, owned=True)

    @classmethod
    def _member(cls, p, dev, st, box, handle):
        self = cls.__new__(cls)
        self._init_from(p, dev, st, box)
        self._set_handle(handle, owned=False)
        return self

    def _init_from(self, p, dev, st, box):
        self._params = p
        dim = p.dim
        self.n = tuple(int(p.n[i]) for i in range(dim))
        self.dim = dim
        self.device = torch.device("cuda", dev)
        self.stream = st
        self.dtype = torch.float64 if p.precision == _lib.FP64 else torch.float32
        self.lam = float(p.lam)
        self.H = math.prod(float(b) / int(m) for b, m in zip(box, self.n))

    def _set_handle(self, h, owned):
        self._h = h
        self._owned = owned
        info = _lib.Info()
        info.struct_size = ctypes.sizeof(_lib.Info)
        check(lib.jgb_plan_info(self._h, ctypes.byref(info)))
        self.info = {f: (list(getattr(info, f)) if f in ("n", "nf", "window") else getattr(info, f))
                     for f, _ in _lib.Info._fields_ if f != "struct_size"}


    # ------------------------------------------------------------ checks
    def _check_grid(self, t, name):
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != self.dtype \
                or tuple(t.shape) != self.n or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor of shape %s on %s"
                             % (name, self.dtype, self.n, self.device))

    # ------------------------------------------------------------ calls
    def potential(self, rho, out=None, energy=True):
        """u = U*rho on the grid and E = (lambda/2) H sum rho u (0-d float64 tensor or None)."""
        self._check_grid(rho, "rho")
        u = torch.empty_like(rho) if out is None else out
        E = torch.empty((), dtype=torch.float64, device=self.device) if energy else None
        check(lib.jgb_potential(self._h, _ptr(rho), _ptr(u), _ptr(E) if energy else None))
        return u, E

    def potential_noalloc(self, rho, out, energy=None):
        """potential() through jgb_potential_noalloc: the library allocates
        nothing during the call (its per-call buffers live in a fixed device
        array shared by every call on the GPU); out (and energy, a 0-d float64
        tensor, if given) must be allocated by the caller."""
        self._check_grid(rho, "rho")
        self._check_grid(out, "out")
        if energy is not None and (energy.dtype != torch.float64 or energy.device != self.device or energy.numel() != 1):
            raise ValueError("energy must be a float64 scalar tensor on %s" % self.device)
        check(lib.jgb_potential_noalloc(self._h, _ptr(rho), _ptr(out), _ptr(energy) if energy is not None else None))
        return out, energy

    def energy(self, rho, out=None):
        self._check_grid(rho, "rho")
        E = torch.empty((), dtype=torch.float64, device=self.device) if out is None else out
        check(lib.jgb_energy(self._h, _ptr(rho), _ptr(E)))
        return E

    def backward(self, grad_u, out=None):
        """Vector-Jacobian product of potential() with respect to rho."""
        self._check_grid(grad_u, "grad_u")
        g = torch.empty_like(grad_u) if out is None else out
        check(lib.jgb_potential_backward(self._h, _ptr(grad_u), _ptr(g)))
        return g

    def _check_psi(self, psi):
        cdt = torch.complex128 if self.dtype == torch.float64 else torch.complex64
        if not isinstance(psi, torch.Tensor) or psi.device != self.device or psi.dtype != cdt \
                or tuple(psi.shape) != self.n or not psi.is_contiguous():
            raise ValueError("psi must be a contiguous %s tensor of shape %s on %s" % (cdt, self.n, self.device))

    def density(self, psi, out=None):
        """rho = |psi|^2 (kernel on the plan's stream)."""
        self._check_psi(psi)
        rho = torch.empty(self.n, dtype=self.dtype, device=self.device) if out is None else out
        check(lib.jgb_density(self._h, _ptr(psi), _ptr(rho)))
        return rho

    def psi_gradient(self, psi, u, gscale=None, factor=2.0, out=None):
        """factor * gscale * lambda * H * u * psi: with factor 2 the PyTorch gradient of E(|psi|^2)."""
        self._check_psi(psi)
        self._check_grid(u, "u")
        grad = torch.empty_like(psi) if out is None else out
        g = None
        if gscale is not None:
            if gscale.dtype != torch.float64 or gscale.device != self.device or gscale.numel() != 1:
                raise ValueError("gscale must be a float64 scalar tensor on %s" % self.device)
            g = _ptr(gscale)
        check(lib.jgb_psi_gradient(self._h, _ptr(psi), _ptr(u), g, float(factor), _ptr(grad)))
        return grad

    def transform(self, rho):
        """rho^ at the half node set (phi index < n_phi/2) in natural order."""
        self._check_grid(rho, "rho")
        cdt = torch.complex128 if self.dtype == torch.float64 else torch.complex64
        out = torch.empty(self.info["n_half"], dtype=cdt, device=self.device)
        check(lib.jgb_transform(self._h, _ptr(rho), _ptr(out)))
        return out

    def nodes(self):
        """(k (M, d), W (M,), c (M,)) of the plan's Fourier quadrature, float64."""
        M = self.info["n_nodes"]
        k = torch.empty((M, self.dim), dtype=torch.float64, device=self.device)
        W = torch.empty(M, dtype=torch.float64, device=self.device)
        c = torch.empty(M, dtype=torch.float64, device=self.device)
        check(lib.jgb_nodes(self._h, _ptr(k), _ptr(W), _ptr(c)))
        return k, W, c

    def timing_begin(self, max_calls):
        """Record per-stage HIP events on the plan's stream for the next max_calls calls."""
        check(lib.jgb_timing_begin(self._h, int(max_calls)))

    def timing_end(self):
        """Synchronise and return ({stage name: average ms}, recorded calls)."""
        ms = (ctypes.c_double * _lib.NUM_STAGES)()
        n = ctypes.c_int()
        check(lib.jgb_timing_end(self._h, ctypes.cast(ms, ctypes.c_void_p), ctypes.cast(ctypes.pointer(n), ctypes.c_void_p)))
        return dict(zip(_lib.STAGE_NAMES, list(ms))), n.value

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and getattr(self, "_owned", True):
            lib.jgb_destroy(h)
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class InteractionEnergy(torch.autograd.Function):
    """E(psi) = (lambda/2) H sum |psi|^2 (U * |psi|^2) with the plan's kernel; the
    backward returns PyTorch's complex gradient 2 g dE/dpsi* = 2 g lambda H u psi.
    Every step (|psi|^2, the convolution, the energy sum, the gradient) is a
    kernel of the library."""

    @staticmethod
    def forward(ctx, psi, plan):
        rho = plan.density(psi)
        u, E = plan.potential(rho)
        ctx.save_for_backward(psi, u)
        ctx.plan = plan
        return E

    @staticmethod
    def backward(ctx, gE):
        psi, u = ctx.saved_tensors
        g = gE.detach().to(torch.float64).contiguous()
        return ctx.plan.psi_gradient(psi, u, gscale=g, factor=2.0), None


# the dipolar energy of the dipole kernel is the same function with a dipole plan
DipolarEnergy = InteractionEnergy


class Batch:
    """Independent densities evaluated by one HIP graph launch.

    members: list of dicts of Plan keyword arguments (n, box, kernel, nodes, eps,
    precision, lam, axis, theta_rule, kmax, split, window, axis2, alpha).  bind() takes the density tensors
    and allocates the outputs; run() evaluates every member."""

    def __init__(self, members, nstreams=4, device=None, stream=None):
        dev = torch.cuda.current_device() if device is None else int(device)
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        arr = (_lib.Params * len(members))()
        boxes = []
        for i, m in enumerate(members):
            kw = dict(eps=1e-10, precision="fp64", lam=1.0, axis=(0.0, 0.0, 1.0), theta_rule="theta", kmax=0.0,
                      autotune=False, split=False, window=(0.0, 0.0), axis2=None, alpha=0.0)
            kw.update(m)
            p, _, _ = _make_params(kw["n"], kw["box"], kw["kernel"], kw["nodes"], kw["eps"], kw["precision"],
                                   kw["lam"], kw["axis"], kw["theta_rule"], kw["kmax"], dev, st, kw["autotune"],
                                   kw["split"], kw["window"], kw["axis2"], kw["alpha"],
                                   **{f: bool(kw.get(f, False)) for f in _FLAG_KWARGS})
            arr[i] = p
            boxes.append(kw["box"])
        h = ctypes.c_void_p()
        check(lib.jgb_batch_create(arr, len(members), int(nstreams), ctypes.byref(h)))
        self._h = h
        self.device = torch.device("cuda", dev)
        self.plans = []
        for i in range(len(members)):
            ph = ctypes.c_void_p()
            check(lib.jgb_batch_plan(self._h, i, ctypes.byref(ph)))
            self.plans.append(Plan._member(arr[i], dev, st, boxes[i], ph))
        self.rho = self.u = self.energies = None

    def bind(self, rhos):
        """Capture the batch for these density tensors; returns (u list, energies tensor)."""
        if len(rhos) != len(self.plans):
            raise ValueError("one density per member")
        for r, p in zip(rhos, self.plans):
            p._check_grid(r, "rho")
        self.rho = list(rhos)
        self.u = [torch.empty_like(r) for r in rhos]
        self.energies = torch.empty(len(rhos), dtype=torch.float64, device=self.device)
        rp = (ctypes.c_void_p * len(rhos))(*[r.data_ptr() for r in self.rho])
        up = (ctypes.c_void_p * len(rhos))(*[u.data_ptr() for u in self.u])
        check(lib.jgb_batch_bind(self._h, rp, up, ctypes.c_void_p(self.energies.data_ptr())))
        return self.u, self.energies

    def run(self):
        check(lib.jgb_batch_run(self._h))
        return self.u, self.energies

    def launches(self):
        """Kernel launches one run() replays (after bind)."""
        n = ctypes.c_int()
        check(lib.jgb_batch_launches(self._h, ctypes.byref(n)))
        return n.value

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            for p in self.plans:
                p._h = ctypes.c_void_p()
            lib.jgb_batch_destroy(h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GPE:
    """Time splitting for i psi_t = [-1/2 Lap + V + beta |psi|^2 + lam Phi] psi,
    Phi = U * |psi|^2 by the potential plan given by the Plan keyword arguments
    (n, box, kernel, nodes, eps, precision, lam, axis, axis2, alpha, theta_rule,
    kmax, split, window).  trap: harmonic frequencies (V = sum trap_j^2 x_j^2 / 2)
    used unless V (a real tensor on the grid) is given; imaginary: the
    ground-state flow with renormalisation.  step() advances psi in place."""

    def __init__(self, n, box, kernel, nodes, dt, beta=0.0, trap=(0.0, 0.0, 0.0), V=None, imaginary=False,
                 device=None, stream=None, **plan_kw):
        kw = dict(eps=1e-10, precision="fp64", lam=1.0, axis=(0.0, 0.0, 1.0), theta_rule="theta", kmax=0.0,
                  autotune=False, split=False, window=(0.0, 0.0), axis2=None, alpha=0.0)
        kw.update(plan_kw)
        p, dev, st = _make_params(n, box, kernel, nodes, kw["eps"], kw["precision"], kw["lam"], kw["axis"],
                                  kw["theta_rule"], kw["kmax"], device, stream, kw["autotune"], kw["split"],
                                  kw["window"], kw["axis2"], kw["alpha"],
                                  **{f: bool(kw.get(f, False)) for f in _FLAG_KWARGS})
        g = _lib.GpeParams()
        g.struct_size = ctypes.sizeof(_lib.GpeParams)
        g.potential = p
        for i in range(3):
            g.trap[i] = float(trap[i]) if i < len(trap) else 0.0
        self.n = tuple(int(v) for v in n)
        self.device = torch.device("cuda", dev)
        self.stream = st
        self.dtype = torch.float64 if p.precision == _lib.FP64 else torch.float32
        self.cdtype = torch.complex128 if self.dtype == torch.float64 else torch.complex64
        self.V = None
        if V is not None:
            if not isinstance(V, torch.Tensor) or V.dtype != self.dtype or tuple(V.shape) != self.n \
                    or V.device != self.device or not V.is_contiguous():
                raise ValueError("V must be a contiguous %s tensor of shape %s on %s" % (self.dtype, self.n, self.device))
            self.V = V
            g.V = ctypes.c_void_p(V.data_ptr())
        g.beta = float(beta)
        g.dt = float(dt)
        g.imaginary = 1 if imaginary else 0
        h = ctypes.c_void_p()
        check(lib.jgb_gpe_create(ctypes.byref(g), ctypes.byref(h)))
        self._h = h

    def _check(self, psi):
        if not isinstance(psi, torch.Tensor) or psi.dtype != self.cdtype or tuple(psi.shape) != self.n \
                or psi.device != self.device or not psi.is_contiguous():
            raise ValueError("psi must be a contiguous %s tensor of shape %s on %s" % (self.cdtype, self.n, self.device))

    def step(self, psi, nsteps=1, graph=True):
        """Advance psi in place by nsteps Strang steps."""
        self._check(psi)
        check(lib.jgb_gpe_step(self._h, _ptr(psi), int(nsteps), 1 if graph else 0))
        return psi

    def energy(self, psi):
        """{norm, kinetic, trap, local, nonlocal, total, mu} of psi (float64 tensor of 7 on the device
        and a dict of floats)."""
        self._check(psi)
        out = torch.empty(7, dtype=torch.float64, device=self.device)
        check(lib.jgb_gpe_energy(self._h, _ptr(psi), _ptr(out)))
        vals = out.cpu().tolist()
        return out, dict(zip(_lib.GPE_ENERGY_NAMES, vals))

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.jgb_gpe_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
