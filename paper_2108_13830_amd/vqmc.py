"""Thin Python binding of libvqmc (the C ABI declared in include/vqmc.h).

Argument marshalling only: tensors are checked (device, dtype, shape,
contiguity) and their device pointers and torch's current HIP stream are
handed to the C entry points of the same names.  Every step of the computation
runs in the library's HIP kernels; if the library is not built, the first call
of any entry point raises (there is no fallback path).
"""
from __future__ import annotations

import ctypes as ct
import os
import dataclasses
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvqmc.so")

PREC_FP32, PREC_BF16, PREC_BF16X3 = 0, 1, 2
PREC_NAMES = {"fp32": PREC_FP32, "bf16": PREC_BF16, "bf16x3": PREC_BF16X3}

SR_AUTO, SR_CHOLESKY, SR_CG, SR_DUAL = 0, 1, 2, 3
ELOC_AUTO, ELOC_DENSE, ELOC_LIGHTCONE = 0, 1, 2

STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported size", 3: "device error",
          4: "workspace too small", 5: "matrix not positive definite",
          6: "conjugate gradients did not converge", 7: "non-finite energies or residual in the SR solve"}
WARN_NOT_CONVERGED = 6


class VqmcError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__("%s: %s (status %d)" % (fn, STATUS.get(status, "?"), status))
        self.status = status


class _Model(ct.Structure):
    _fields_ = [("L", ct.c_int32), ("channels", ct.c_int32), ("n_layers", ct.c_int32),
                ("activation", ct.c_int32), ("J1", ct.c_double), ("J2", ct.c_double),
                ("marshall", ct.c_int32), ("conv_prec", ct.c_int32), ("eloc_mode", ct.c_int32),
                ("symmetry", ct.c_int32)]


class _SrOpts(ct.Structure):
    _fields_ = [("method", ct.c_int32), ("s_prec", ct.c_int32), ("eps", ct.c_double),
                ("tol", ct.c_double), ("max_iter", ct.c_int32)]


class _SrInfo(ct.Structure):
    _fields_ = [("e_mean", ct.c_double), ("e_var", ct.c_double), ("iters", ct.c_int32),
                ("rel_residual", ct.c_double)]


@dataclass(frozen=True)
class Model:
    """Lattice L x L, C channels, n C->C layers after the lift, couplings,
    Marshall sign on/off, the precision of the forward convolutions, the
    local-energy method and the rotation symmetrisation on/off."""
    L: int
    C: int
    n: int
    J1: float = 1.0
    J2: float = 0.5
    marshall: int = 1
    prec: int = PREC_FP32
    eloc: int = ELOC_AUTO
    symmetry: int = 0

    def c(self) -> _Model:
        return _Model(self.L, self.C, self.n, 0, self.J1, self.J2, self.marshall, self.prec, self.eloc,
                      self.symmetry)

    def with_prec(self, prec) -> "Model":
        p = PREC_NAMES[prec] if isinstance(prec, str) else prec
        return dataclasses.replace(self, prec=p)

    def with_eloc(self, eloc) -> "Model":
        return dataclasses.replace(self, eloc=eloc)

    def with_symmetry(self, symmetry: int = 1) -> "Model":
        return dataclasses.replace(self, symmetry=symmetry)

    @property
    def N(self) -> int:
        return self.L * self.L


@dataclass(frozen=True)
class SrOpts:
    method: int = SR_AUTO
    s_prec: int = 1
    eps: float = 1e-4
    tol: float = 1e-8
    max_iter: int = 200

    def c(self) -> _SrOpts:
        return _SrOpts(self.method, self.s_prec, self.eps, self.tol, self.max_iter)


_lib = None

# every entry point of include/vqmc.h: (name, restype, argtypes)
_VP = ct.c_void_p
SIGNATURES = [
    ("vqmc_num_params", ct.c_int64, [ct.POINTER(_Model)]),
    ("vqmc_status_string", ct.c_char_p, [ct.c_int]),
    ("vqmc_sample", ct.c_int, [ct.POINTER(_Model), _VP, _VP, _VP, ct.c_int32, ct.c_int32,
                               ct.c_uint64, ct.c_uint64, ct.c_int32, _VP, _VP]),
    ("vqmc_log_psi", ct.c_int, [ct.POINTER(_Model), _VP, _VP, ct.c_int32, _VP, _VP, _VP]),
    ("vqmc_local_energy", ct.c_int, [ct.POINTER(_Model), _VP, _VP, ct.c_int32, _VP, _VP, _VP,
                                     ct.c_size_t, _VP]),
    ("vqmc_local_energy_noalloc", ct.c_int, [ct.POINTER(_Model), _VP, _VP, ct.c_int32, _VP, _VP, _VP]),
    ("vqmc_local_energy_method", ct.c_int, [ct.POINTER(_Model), ct.POINTER(ct.c_int32)]),
    ("vqmc_local_energy_workspace", ct.c_int, [ct.POINTER(_Model), ct.c_int32,
                                               ct.POINTER(ct.c_size_t)]),
    ("vqmc_log_derivs_workspace", ct.c_int, [ct.POINTER(_Model), ct.c_int32,
                                             ct.POINTER(ct.c_size_t)]),
    ("vqmc_log_derivs", ct.c_int, [ct.POINTER(_Model), _VP, _VP, ct.c_int32, _VP, ct.c_int64,
                                   _VP, ct.c_size_t, _VP]),
    ("vqmc_sr_workspace", ct.c_int, [ct.c_int32, ct.c_int64, ct.POINTER(_SrOpts),
                                     ct.POINTER(ct.c_size_t)]),
    ("vqmc_sr_solve", ct.c_int, [_VP, ct.c_int64, _VP, ct.c_int32, ct.c_int64,
                                 ct.POINTER(_SrOpts), _VP, _VP, _VP, ct.c_size_t,
                                 ct.POINTER(_SrInfo), _VP]),
    ("vqmc_vmc_step", ct.c_int, [ct.POINTER(_Model), _VP, _VP, ct.c_int32, ct.c_int32, ct.c_uint64,
                                 ct.c_uint64, ct.c_int32, ct.POINTER(_SrOpts), ct.c_double, _VP, _VP,
                                 ct.c_size_t, ct.POINTER(_SrInfo), _VP]),
    ("vqmc_vmc_step_workspace", ct.c_int, [ct.POINTER(_Model), ct.c_int32, ct.POINTER(_SrOpts),
                                           ct.POINTER(ct.c_size_t)]),
    # measurement helper (include/vqmc_probe.h)
    ("vqmc_probe_mfma", ct.c_int, [ct.c_int, ct.c_int, ct.c_int, _VP, _VP, ct.POINTER(ct.c_double), _VP]),
]


def lib():
    """The loaded libvqmc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libvqmc.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2108_13830_amd.build)")
        L = ct.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    """Names of SIGNATURES that the built library exports."""
    L = ct.CDLL(LIB_PATH)
    return [name for name, _, _ in SIGNATURES if hasattr(L, name)]


def _check(fn, rc, allow=()):
    if rc != 0 and rc not in allow:
        raise VqmcError(fn, rc)
    return rc


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ct.c_void_p(0 if t is None else t.data_ptr())


def _dev(t, dtype, name, shape=None):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))


def num_params(m: Model) -> int:
    mc = m.c()
    return int(lib().vqmc_num_params(ct.byref(mc)))


def vqmc_log_psi(m: Model, theta, spins, out=None, sign=None):
    """log|W_CNN| (double [B]) and, if sign is given, the Marshall sign."""
    B = spins.shape[0]
    _dev(theta, torch.float32, "theta", (num_params(m),))
    _dev(spins, torch.int8, "spins", (B, m.N))
    if out is None:
        out = torch.empty(B, dtype=torch.float64, device=spins.device)
    _dev(out, torch.float64, "out", (B,))
    _dev(sign, torch.int8, "sign", (B,))
    mc = m.c()
    _check("vqmc_log_psi", lib().vqmc_log_psi(ct.byref(mc), _ptr(theta), _ptr(spins), B,
                                              _ptr(out), _ptr(sign), _stream()))
    return out


def local_energy_method(m: Model) -> int:
    """ELOC_DENSE or ELOC_LIGHTCONE: the method the library uses for m."""
    mc = m.c()
    r = ct.c_int32(0)
    _check("vqmc_local_energy_method", lib().vqmc_local_energy_method(ct.byref(mc), ct.byref(r)))
    return r.value


def local_energy_workspace(m: Model, B: int) -> int:
    mc = m.c()
    n = ct.c_size_t(0)
    _check("vqmc_local_energy_workspace", lib().vqmc_local_energy_workspace(ct.byref(mc), B,
                                                                            ct.byref(n)))
    return n.value


def vqmc_local_energy(m: Model, theta, spins, out=None, flags=None, workspace=None):
    B = spins.shape[0]
    _dev(theta, torch.float32, "theta", (num_params(m),))
    _dev(spins, torch.int8, "spins", (B, m.N))
    if out is None:
        out = torch.empty(B, dtype=torch.float64, device=spins.device)
    _dev(out, torch.float64, "out", (B,))
    _dev(flags, torch.int32, "flags", (B,))
    ws = local_energy_workspace(m, B)
    if workspace is None and ws > 0:
        workspace = torch.empty(ws, dtype=torch.uint8, device=spins.device)
    mc = m.c()
    _check("vqmc_local_energy", lib().vqmc_local_energy(
        ct.byref(mc), _ptr(theta), _ptr(spins), B, _ptr(out), _ptr(flags), _ptr(workspace),
        0 if workspace is None else workspace.numel(), _stream()))
    return out


def vqmc_local_energy_noalloc(m: Model, theta, spins, out=None, flags=None):
    """The local energy in the dense evaluation with no workspace: the
    library keeps the packed weights in its own device array (for callers
    that cannot allocate device memory)."""
    B = spins.shape[0]
    _dev(theta, torch.float32, "theta", (num_params(m),))
    _dev(spins, torch.int8, "spins", (B, m.N))
    if out is None:
        out = torch.empty(B, dtype=torch.float64, device=spins.device)
    _dev(out, torch.float64, "out", (B,))
    _dev(flags, torch.int32, "flags", (B,))
    mc = m.c()
    _check("vqmc_local_energy_noalloc", lib().vqmc_local_energy_noalloc(
        ct.byref(mc), _ptr(theta), _ptr(spins), B, _ptr(out), _ptr(flags), _stream()))
    return out


def vqmc_sample(m: Model, theta, spins, n_sweeps: int, seed: int, counter_base: int = 0,
                proposal: int = 0, log_psi=None, n_accepted=None):
    """Runs the chains in place on spins; returns spins."""
    B = spins.shape[0]
    _dev(theta, torch.float32, "theta", (num_params(m),))
    _dev(spins, torch.int8, "spins", (B, m.N))
    _dev(log_psi, torch.float64, "log_psi", (B,))
    _dev(n_accepted, torch.int32, "n_accepted", (B,))
    mc = m.c()
    _check("vqmc_sample", lib().vqmc_sample(ct.byref(mc), _ptr(theta), _ptr(spins), _ptr(log_psi),
                                            B, n_sweeps, seed, counter_base, proposal,
                                            _ptr(n_accepted), _stream()))
    return spins


def log_derivs_workspace(m: Model, B: int) -> int:
    mc = m.c()
    n = ct.c_size_t(0)
    _check("vqmc_log_derivs_workspace", lib().vqmc_log_derivs_workspace(ct.byref(mc), B,
                                                                        ct.byref(n)))
    return n.value


def vqmc_log_derivs(m: Model, theta, spins, O=None, workspace=None):
    """O[b][k] = d log|psi(sigma_b)| / d theta_k (float32 [B][P])."""
    B = spins.shape[0]
    P = num_params(m)
    _dev(theta, torch.float32, "theta", (P,))
    _dev(spins, torch.int8, "spins", (B, m.N))
    if O is None:
        O = torch.empty((B, P), dtype=torch.float32, device=spins.device)
    if O.dim() != 2 or O.shape[0] != B or O.shape[1] < P or O.stride(1) != 1:
        raise ValueError("O must be [B][ldO] with ldO >= P and unit column stride")
    ws = log_derivs_workspace(m, B)
    if workspace is None:
        workspace = torch.empty(max(ws, 1), dtype=torch.uint8, device=spins.device)
    mc = m.c()
    _check("vqmc_log_derivs", lib().vqmc_log_derivs(ct.byref(mc), _ptr(theta), _ptr(spins), B,
                                                    _ptr(O), O.stride(0), _ptr(workspace),
                                                    workspace.numel(), _stream()))
    return O


def sr_workspace(B: int, P: int, opts: SrOpts) -> int:
    oc = opts.c()
    n = ct.c_size_t(0)
    _check("vqmc_sr_workspace", lib().vqmc_sr_workspace(B, P, ct.byref(oc), ct.byref(n)))
    return n.value


def vqmc_sr_solve(O, e_loc, opts: SrOpts = SrOpts(), P: int | None = None, delta=None, F=None,
                  workspace=None, want_info: bool = True):
    """Solve (S + eps I) delta = F; returns (delta, F, info dict or None)."""
    B = O.shape[0]
    P = O.shape[1] if P is None else P
    if O.dim() != 2 or O.stride(1) != 1 or O.dtype != torch.float32 or not O.is_cuda:
        raise ValueError("O must be a float32 GPU matrix with unit column stride")
    _dev(e_loc, torch.float64, "e_loc", (B,))
    if delta is None:
        delta = torch.empty(P, dtype=torch.float64, device=O.device)
    if F is None:
        F = torch.empty(P, dtype=torch.float64, device=O.device)
    _dev(delta, torch.float64, "delta", (P,))
    _dev(F, torch.float64, "F", (P,))
    ws = sr_workspace(B, P, opts)
    if workspace is None:
        workspace = torch.empty(max(ws, 1), dtype=torch.uint8, device=O.device)
    oc = opts.c()
    info = _SrInfo()
    rc = lib().vqmc_sr_solve(_ptr(O), O.stride(0), _ptr(e_loc), B, P, ct.byref(oc), _ptr(delta),
                             _ptr(F), _ptr(workspace), workspace.numel(),
                             ct.byref(info) if want_info else None, _stream())
    _check("vqmc_sr_solve", rc, allow=(WARN_NOT_CONVERGED,))
    d = None
    if want_info:
        d = dict(e_mean=info.e_mean, e_var=info.e_var, iters=info.iters,
                 rel_residual=info.rel_residual, converged=(rc == 0))
    return delta, F, d


def vmc_step_workspace(m: Model, B: int, opts: SrOpts) -> int:
    mc, oc = m.c(), opts.c()
    n = ct.c_size_t(0)
    _check("vqmc_vmc_step_workspace", lib().vqmc_vmc_step_workspace(ct.byref(mc), B, ct.byref(oc),
                                                                    ct.byref(n)))
    return n.value


def vqmc_vmc_step(m: Model, theta, spins, n_sweeps: int, seed: int, counter_base: int, lr: float,
                  opts: SrOpts = SrOpts(), proposal: int = 0, e_loc=None, workspace=None,
                  want_info: bool = True):
    """One optimisation iteration in place on theta and spins: sampling,
    E_s, O_s, the SR solve and theta -= lr * delta.  Returns the info dict
    (energy mean/variance, SR report) or None."""
    B = spins.shape[0]
    _dev(theta, torch.float32, "theta", (num_params(m),))
    _dev(spins, torch.int8, "spins", (B, m.N))
    _dev(e_loc, torch.float64, "e_loc", (B,))
    ws = vmc_step_workspace(m, B, opts)
    if workspace is None:
        workspace = torch.empty(max(ws, 1), dtype=torch.uint8, device=spins.device)
    mc, oc = m.c(), opts.c()
    info = _SrInfo()
    rc = lib().vqmc_vmc_step(ct.byref(mc), _ptr(theta), _ptr(spins), B, n_sweeps, seed & (2**64 - 1),
                             counter_base, proposal, ct.byref(oc), lr, _ptr(e_loc), _ptr(workspace),
                             workspace.numel(), ct.byref(info) if want_info else None, _stream())
    _check("vqmc_vmc_step", rc, allow=(WARN_NOT_CONVERGED,))
    if not want_info:
        return None
    return dict(e_mean=info.e_mean, e_var=info.e_var, iters=info.iters, rel_residual=info.rel_residual,
                converged=(rc == 0))


PROBE_KINDS = {"bf16": 0, "bf16x3": 0, "fp32": 1, "fp64": 2}


def probe_mfma(kind: str, iters: int = 20000, blocks: int = 2048) -> float:
    """Achievable matrix-core TFLOP/s of one instruction kind on the current
    GPU (vqmc_probe_mfma timed with HIP events on the current stream; one
    warm-up launch)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    x = torch.linspace(0.5, 1.5, 128, dtype=torch.float32, device=dev)
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    fl = ct.c_double(0.0)
    k = PROBE_KINDS[kind]
    _check("vqmc_probe_mfma", lib().vqmc_probe_mfma(k, 10, blocks, _ptr(x), _ptr(out), None, _stream()))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _check("vqmc_probe_mfma", lib().vqmc_probe_mfma(k, iters, blocks, _ptr(x), _ptr(out), ct.byref(fl),
                                                     _stream()))
    e1.record()
    torch.cuda.synchronize()
    return fl.value / (e0.elapsed_time(e1) / 1e3) / 1e12


class LogPsi(torch.autograd.Function):
    """log|psi(sigma)| as a differentiable function of theta.  The forward
    calls vqmc_log_psi; the backward calls vqmc_log_derivs (the per-sample
    O_k) and contracts with the incoming gradient."""

    @staticmethod
    def forward(ctx, theta, spins, m):
        ctx.save_for_backward(theta, spins)
        ctx.m = m
        return vqmc_log_psi(m, theta.detach(), spins)

    @staticmethod
    def backward(ctx, g):
        theta, spins = ctx.saved_tensors
        O = vqmc_log_derivs(ctx.m, theta.detach(), spins)
        return (g.to(torch.float64) @ O.to(torch.float64)).to(theta.dtype), None, None


def log_psi(theta, spins, m: Model):
    return LogPsi.apply(theta, spins, m)
