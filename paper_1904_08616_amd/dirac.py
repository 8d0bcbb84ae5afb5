"""PyTorch-facing binding of libdirac.

Only argument marshalling lives here: every arithmetic step of the
operator, the solver and the gradients runs in the library's HIP kernels.
PyTorch provides device memory (uint8 buffers in the library's internal
layout, complex128 tensors in the canonical layout) and the current stream.

Canonical layouts (as in include/dirac.h):
  links   U   : complex128 [T, Z, Y, X, 4, 3, 3]
  spinors psi : complex128 [T, Z, Y, X, 4, 3]  or  [nrhs, T, Z, Y, X, 4, 3]
  force   F   : complex128 [T, Z, Y, X, 4, 3, 3]
``dims`` is always (Lx, Ly, Lz, Lt).
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi as abi

PRECISIONS = {"f64": abi.F64, "f32": abi.F32, "f16s": abi.F16S, "bf16s": abi.BF16S}


def _prec(p):
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return C.c_void_p(0)
    if not t.is_cuda:
        raise ValueError("expected a CUDA (HIP) tensor")
    return C.c_void_p(t.data_ptr())


def _cuda_c128(t, shape, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128):
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.contiguous()


class Operator:
    """One instance of eq. (1): geometry, quark mass, precision, link storage, nrhs."""

    def __init__(self, dims, m_q, prec="f64", link=18, nrhs=1):
        self.dims = tuple(int(d) for d in dims)
        self.m_q = float(m_q)
        self.prec = _prec(prec)
        self.link = int(link)
        self.nrhs = int(nrhs)
        self.op = abi.make_op(self.dims, self.prec, self.link, self.nrhs, self.m_q)
        self.lib = abi.load()

    # ---------------------------------------------------------------- shapes
    @property
    def site_shape(self):
        lx, ly, lz, lt = self.dims
        return (lt, lz, ly, lx)

    @property
    def volume(self):
        return int(np.prod(self.dims))

    def spinor_shape(self):
        s = self.site_shape + (4, 3)
        return s if self.nrhs == 1 else (self.nrhs,) + s

    def gauge_shape(self):
        return self.site_shape + (4, 3, 3)

    def like(self, prec=None, link=None, nrhs=None, m_q=None):
        return Operator(self.dims, self.m_q if m_q is None else m_q, self.prec if prec is None else prec,
                        self.link if link is None else link, self.nrhs if nrhs is None else nrhs)

    def spinor_bytes(self):
        return int(abi.check(self.lib.dirac_spinor_bytes(C.byref(self.op))))

    def gauge_bytes(self):
        return int(abi.check(self.lib.dirac_gauge_bytes(C.byref(self.op))))

    def empty_spinor(self, device="cuda"):
        return torch.empty(self.spinor_bytes(), dtype=torch.uint8, device=device)

    def empty_gauge(self, device="cuda"):
        return torch.empty(self.gauge_bytes(), dtype=torch.uint8, device=device)

    # ---------------------------------------------------------------- layout
    def pack_gauge(self, U, out=None):
        U = _cuda_c128(U, self.gauge_shape(), "U")
        out = self.empty_gauge(U.device) if out is None else out
        abi.check(self.lib.dirac_pack_gauge(C.byref(self.op), _ptr(U), _ptr(out), _stream()))
        return out

    def pack_spinor(self, psi, out=None):
        psi = _cuda_c128(psi, self.spinor_shape(), "psi")
        out = self.empty_spinor(psi.device) if out is None else out
        abi.check(self.lib.dirac_pack_spinor(C.byref(self.op), _ptr(psi), _ptr(out), _stream()))
        return out

    def unpack_spinor(self, buf, out=None):
        if out is None:
            out = torch.empty(self.spinor_shape(), dtype=torch.complex128, device=buf.device)
        abi.check(self.lib.dirac_unpack_spinor(C.byref(self.op), _ptr(buf), _ptr(out), _stream()))
        return out

    def convert(self, buf, dst_op, out=None):
        out = dst_op.empty_spinor(buf.device) if out is None else out
        abi.check(self.lib.dirac_convert_spinor(C.byref(self.op), _ptr(buf), C.byref(dst_op.op), _ptr(out),
                                                _stream()))
        return out

    # -------------------------------------------------------------- operator
    def apply(self, U_int, psi_int, out=None, dagger=False):
        out = self.empty_spinor(psi_int.device) if out is None else out
        fn = self.lib.dirac_dagger_apply if dagger else self.lib.dirac_apply
        abi.check(fn(C.byref(self.op), _ptr(U_int), _ptr(psi_int), _ptr(out), _stream()))
        return out

    def schur(self, U_int, in_int, out=None, dagger=False):
        """Even-odd Schur complement D_hat (or D_hat^dagger) on the even plane
        of ``in_int``; the odd plane of ``out`` is overwritten (scratch)."""
        out = self.empty_spinor(in_int.device) if out is None else out
        abi.check(self.lib.dirac_schur_apply(C.byref(self.op), _ptr(U_int), _ptr(in_int), _ptr(out),
                                             1 if dagger else 0, _stream()))
        return out

    def mdagm(self, U_int, psi_int, out=None, tmp=None):
        out = self.empty_spinor(psi_int.device) if out is None else out
        tmp = self.empty_spinor(psi_int.device) if tmp is None else tmp
        abi.check(self.lib.dirac_mdagm_apply(C.byref(self.op), _ptr(U_int), _ptr(psi_int), _ptr(tmp),
                                             _ptr(out), _stream()))
        return out

    def dot_workspace(self, device="cuda"):
        """A device workspace for ``dot`` (kept by the operator and reused)."""
        need = int(abi.check(self.lib.dirac_field_dot_workspace_bytes(C.byref(self.op))))
        ws = getattr(self, "_dot_ws", None)
        if ws is None or ws.numel() < need or ws.device != torch.device(device):
            ws = torch.empty(need, dtype=torch.uint8, device=device)
            self._dot_ws = ws
        return ws

    def dot(self, a, b, workspace=None):
        out = (C.c_double * (2 * self.nrhs))()
        ws = self.dot_workspace(a.device) if workspace is None else workspace
        abi.check(self.lib.dirac_field_dot(C.byref(self.op), _ptr(a), _ptr(b), _ptr(ws), C.c_int64(ws.numel()),
                                           out, _stream()))
        v = np.frombuffer(out, dtype=np.float64).copy()
        return v[0::2] + 1j * v[1::2]

    def dot_noalloc(self, a, b):
        """``dot`` through dirac_field_dot_noalloc (the library's fixed
        scratch array; no workspace)."""
        out = (C.c_double * (2 * self.nrhs))()
        abi.check(self.lib.dirac_field_dot_noalloc(C.byref(self.op), _ptr(a), _ptr(b), out, _stream()))
        v = np.frombuffer(out, dtype=np.float64).copy()
        return v[0::2] + 1j * v[1::2]

    def axpy(self, a, x, y):
        a = complex(a)
        abi.check(self.lib.dirac_field_axpy(C.byref(self.op), a.real, a.imag, _ptr(x), _ptr(y), _stream()))
        return y

    def force(self, g_int, psi_int, coeff=1.0, out=None, accumulate=False):
        if out is None:
            out = torch.zeros(self.gauge_shape(), dtype=torch.complex128, device=g_int.device)
        abi.check(self.lib.dirac_force(C.byref(self.op), _ptr(g_int), _ptr(psi_int), _ptr(out), float(coeff),
                                       1 if accumulate else 0, _stream()))
        return out

    # ---------------------------------------------------------------- tuning
    def autotune(self, U_int, psi_int, chi_int):
        abi.check(self.lib.dirac_autotune(C.byref(self.op), _ptr(U_int), _ptr(psi_int), _ptr(chi_int),
                                          _stream()))
        return self.launch_config()

    def launch_config(self):
        out = abi.DiracLaunch()
        abi.check(self.lib.dirac_launch_config(C.byref(self.op), C.byref(out)))
        return out.as_dict()

    def set_launch_config(self, block_sites=128, rhs_per_thread=1, xcd_remap=1, lds=0, nt_store=0,
                          tile_y=1, tile_z=1, t_chunk=1):
        cfg = abi.DiracLaunch(block_sites, rhs_per_thread, xcd_remap, nt_store, lds, tile_y, tile_z, t_chunk, 0)
        abi.check(self.lib.dirac_set_launch_config(C.byref(self.op), C.byref(cfg)))


# -------------------------------------------------------------------- CG ----

def cg(op_hi, U_hi, eta_int, x_int=None, tol=1e-10, max_iter=100000, inner_prec="f64", U_lo=None,
       inner_delta=0.0, inner_kmax=0, check_every=0, workspace=None, allow_failure=False, single_launch=0):
    """Solve D^dag D x = eta with cg_solve.  Returns (x_int, [stats dict per RHS]).
    single_launch: 0 automatic, 1 / -1 force the single-launch iteration on / off."""
    lib = abi.load()
    prm = abi.CgParams(float(tol), int(max_iter), _prec(inner_prec), float(inner_delta), int(inner_kmax),
                       int(check_every), int(single_launch), 0)
    if x_int is None:
        x_int = torch.zeros_like(eta_int)
    need = int(abi.check(lib.cg_workspace_bytes(C.byref(op_hi.op), C.byref(prm))))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=eta_int.device)
    stats = (abi.CgStats * op_hi.nrhs)()
    rc = lib.cg_solve(C.byref(op_hi.op), _ptr(U_hi), _ptr(U_lo), _ptr(eta_int), _ptr(x_int), _ptr(workspace),
                      C.c_int64(workspace.numel()), C.byref(prm), stats, _stream())
    abi.check(rc, allow=(abi.ENOCONV, abi.EBREAKDOWN) if allow_failure else ())
    return x_int, [s.as_dict() for s in stats]


def cg_eo(op_hi, U_hi, b_int, x_int=None, tol=1e-10, max_iter=100000, inner_prec="f64", U_lo=None,
          inner_delta=0.0, inner_kmax=0, check_every=0, workspace=None, allow_failure=False, dagger=False):
    """Solve D x = b (D^dag x = b with dagger) through the even-odd Schur complement
    (cg_solve_eo).  Returns (x_int, [stats dict per RHS]); true_rel_res is
    ||b - D x|| / ||b||."""
    lib = abi.load()
    prm = abi.CgParams(float(tol), int(max_iter), _prec(inner_prec), float(inner_delta), int(inner_kmax),
                       int(check_every))
    if x_int is None:
        x_int = torch.zeros_like(b_int)
    need = int(abi.check(lib.cg_workspace_bytes_eo(C.byref(op_hi.op), C.byref(prm))))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=b_int.device)
    stats = (abi.CgStats * op_hi.nrhs)()
    rc = lib.cg_solve_eo(C.byref(op_hi.op), _ptr(U_hi), _ptr(U_lo), _ptr(b_int), _ptr(x_int), _ptr(workspace),
                         C.c_int64(workspace.numel()), C.byref(prm), 1 if dagger else 0, stats, _stream())
    abi.check(rc, allow=(abi.ENOCONV, abi.EBREAKDOWN) if allow_failure else ())
    return x_int, [s.as_dict() for s in stats]


# -------------------------------------------------------- batched lattices ----

def bandwidth_probe(kind, src, dst, nbytes):
    """Bandwidth reference kernel (dirac_bandwidth_probe): 'copy', 'read' or 'write'."""
    k = {"copy": 0, "read": 1, "write": 2}[kind]
    abi.check(abi.load().dirac_bandwidth_probe(k, _ptr(src), _ptr(dst), C.c_int64(nbytes), _stream()))


def _ptr_array(ts):
    return (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


def multi_apply(ops, Us, psis, chis, dagger=False):
    lib = abi.load()
    arr = (abi.DiracOp * len(ops))(*[o.op for o in ops])
    abi.check(lib.dirac_multi_apply(len(ops), arr, _ptr_array(Us), _ptr_array(psis), _ptr_array(chis),
                                    1 if dagger else 0, _stream()))
    return chis


class MultiPlan:
    """dirac_multi_apply captured once in a hipGraph; ``launch()`` replays it."""

    def __init__(self, ops, Us, psis, chis, dagger=False):
        self.lib = abi.load()
        self._keep = (list(Us), list(psis), list(chis))  # buffers must outlive the plan
        arr = (abi.DiracOp * len(ops))(*[o.op for o in ops])
        h = C.c_void_p()
        abi.check(self.lib.dirac_multi_plan_create(len(ops), arr, _ptr_array(Us), _ptr_array(psis),
                                                   _ptr_array(chis), 1 if dagger else 0, _stream(),
                                                   C.byref(h)))
        self.handle = h

    def launch(self):
        abi.check(self.lib.dirac_plan_launch(self.handle, _stream()))

    def close(self):
        if self.handle:
            self.lib.dirac_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------- canonical helpers ----

def apply_dirac(U, psi, m_q, prec="f64", link=18, dagger=False):
    """chi = D psi (or D^dag psi) on canonical complex128 CUDA tensors."""
    nrhs = 1 if psi.dim() == 6 else psi.shape[0]
    lt, lz, ly, lx = U.shape[:4]
    op = Operator((lx, ly, lz, lt), m_q, prec, link, nrhs)
    Ui = op.pack_gauge(U)
    pi = op.pack_spinor(psi)
    return op.unpack_spinor(op.apply(Ui, pi, dagger=dagger))


class DiracApply(torch.autograd.Function):
    """chi = D(U) psi (eq. (1)), float64, 18-real links.

    Backward (PyTorch's complex convention grad = dL/dRe + i dL/dIm):
      grad_psi = D^dag grad_chi
      grad_U   = link force: 1/2 [ sum_a g(n)_a (P^- psi(n+mu))_a^dag + sum_a (P^+ psi(n))_a g(n+mu)_a^dag ]
    both evaluated by the library's kernels.
    """

    @staticmethod
    def forward(ctx, U, psi, m_q):
        lt, lz, ly, lx = U.shape[:4]
        op = Operator((lx, ly, lz, lt), m_q, "f64", 18, 1)
        Ui = op.pack_gauge(U.detach())
        pi = op.pack_spinor(psi.detach())
        chi = op.unpack_spinor(op.apply(Ui, pi))
        ctx.op = op
        ctx.save_for_backward(Ui, pi)
        return chi

    @staticmethod
    def backward(ctx, g):
        op = ctx.op
        Ui, pi = ctx.saved_tensors
        gi = op.pack_spinor(g.contiguous())
        gU = gpsi = None
        if ctx.needs_input_grad[1]:
            gpsi = op.unpack_spinor(op.apply(Ui, gi, dagger=True))
        if ctx.needs_input_grad[0]:
            gU = op.force(gi, pi, coeff=1.0)
        return gU, gpsi, None


class DSolve(torch.autograd.Function):
    """x = D^{-1} b (the propagator) by the library's even-odd solve, to a
    float64 residual ||b - D x|| / ||b|| < tol; inner_prec "f32", "f16s" or
    "bf16s" runs its CG as Algorithm 1 with that inner format (the tolerance
    is still met in float64).

    Backward: lambda = D^{-dag} grad_x (the even-odd solve with D^dagger, same
    inner format), grad_b = lambda, grad_U = -force(lambda, x).
    """

    @staticmethod
    def forward(ctx, U, b, m_q, tol=1e-12, max_iter=100000, inner_prec="f64"):
        lt, lz, ly, lx = U.shape[:4]
        op = Operator((lx, ly, lz, lt), m_q, "f64", 18, 1)
        Ui = op.pack_gauge(U.detach())
        Ul = None
        if inner_prec != "f64":
            Ul = op.like(prec=inner_prec, link=18 if inner_prec == "f32" else 12).pack_gauge(U.detach())
        bi = op.pack_spinor(b.detach())
        x, st = cg_eo(op, Ui, bi, tol=tol, max_iter=max_iter, inner_prec=inner_prec, U_lo=Ul)
        ctx.op, ctx.tol, ctx.max_iter, ctx.inner, ctx.Ul = op, tol, max_iter, inner_prec, Ul
        ctx.save_for_backward(Ui, x)
        ctx.stats = st
        return op.unpack_spinor(x)

    @staticmethod
    def backward(ctx, gx):
        op = ctx.op
        Ui, x = ctx.saved_tensors
        gi = op.pack_spinor(gx.contiguous())
        lam, _ = cg_eo(op, Ui, gi, tol=ctx.tol, max_iter=ctx.max_iter, inner_prec=ctx.inner, U_lo=ctx.Ul,
                       dagger=True)
        gU = gb = None
        if ctx.needs_input_grad[1]:
            gb = op.unpack_spinor(lam)
        if ctx.needs_input_grad[0]:
            gU = op.force(lam, x, coeff=-1.0)
        return gU, gb, None, None, None, None


class DdagDSolve(torch.autograd.Function):
    """X = (D^dag D)^{-1} phi by the library's float64 CG.

    Backward: lambda = (D^dag D)^{-1} grad_X (a second solve), grad_phi = lambda,
    grad_U = -[ force(D X, lambda) + force(D lambda, X) ].
    """

    @staticmethod
    def forward(ctx, U, phi, m_q, tol=1e-12, max_iter=100000):
        lt, lz, ly, lx = U.shape[:4]
        op = Operator((lx, ly, lz, lt), m_q, "f64", 18, 1)
        Ui = op.pack_gauge(U.detach())
        eta = op.pack_spinor(phi.detach())
        x, st = cg(op, Ui, eta, tol=tol, max_iter=max_iter)
        ctx.op, ctx.tol, ctx.max_iter = op, tol, max_iter
        ctx.save_for_backward(Ui, x)
        ctx.stats = st
        return op.unpack_spinor(x)

    @staticmethod
    def backward(ctx, gX):
        op = ctx.op
        Ui, x = ctx.saved_tensors
        gi = op.pack_spinor(gX.contiguous())
        lam, _ = cg(op, Ui, gi, tol=ctx.tol, max_iter=ctx.max_iter)
        gU = gphi = None
        if ctx.needs_input_grad[1]:
            gphi = op.unpack_spinor(lam)
        if ctx.needs_input_grad[0]:
            dx = op.apply(Ui, x)
            dl = op.apply(Ui, lam)
            gU = op.force(dx, lam, coeff=-1.0)
            op.force(dl, x, coeff=-1.0, out=gU, accumulate=True)
        return gU, gphi, None, None, None
