"""Python objects over the C ABI: Geometry, Plan and the autograd Function.

Only argument marshalling happens here; every numerical step runs in the HIP
kernels of libcosim.so.  Device arrays are torch tensors on the current HIP
device, work is enqueued on torch's current stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import numpy as np
import torch

from ._lib import check, load_library

FP64, FP32, BF16X3 = 0, 1, 2
LOSS_MAG, LOSS_COMPLEX, LOSS_RATIO = 0, 1, 2
SYS_BAD_INPUT, SYS_SINGULAR, SYS_NONFINITE, SYS_NEGATIVE_C = 1, 2, 4, 8

_PREC_NAMES = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}


def precision_code(p) -> int:
    if isinstance(p, str):
        return _PREC_NAMES[p.lower()]
    return int(p)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype: torch.dtype, shape, name: str) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise TypeError(f"{name} must live on the GPU (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _host(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


class Geometry:
    """Closed polygonal loops (see include/cosim.h, cosim_geometry_create)."""

    def __init__(self, verts, seg_off, wire_a, R):
        self._lib = load_library()
        self.verts = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 3)
        self.seg_off = np.ascontiguousarray(seg_off, dtype=np.int32)
        n = int(self.seg_off.shape[0] - 1)
        self.wire_a = np.ascontiguousarray(np.broadcast_to(wire_a, (n,)), dtype=np.float64)
        self.R = np.ascontiguousarray(np.broadcast_to(R, (n,)), dtype=np.float64)
        h = ctypes.c_void_p()
        check(self._lib.cosim_geometry_create(n, _host(self.seg_off), _host(self.verts),
                                              _host(self.wire_a), _host(self.R), ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_workload(cls, g) -> "Geometry":
        return cls(g.verts, g.seg_off, g.wire_a, g.R)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    @property
    def n(self) -> int:
        v = ctypes.c_int()
        check(self._lib.cosim_geometry_size(self._h, ctypes.byref(v), None))
        return v.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.cosim_geometry_destroy(h)
            self._h = None


class Plan:
    """Assembled operators G, M, Phi for one geometry and point set.

    precisions: None for every precision, or an iterable of precisions whose
    copies of G the plan keeps (cosim_assemble_ex).  component: the Cartesian
    component of the field that G holds, 0 (x), 1 (y) or 2 (z)
    (cosim_assemble_component)."""

    def __init__(self, geom: Geometry, pts: torch.Tensor, bext_z: float = 1e-6,
                 precisions=None, component: int = 2):
        self._lib = load_library()
        P = int(pts.shape[0])
        ptr = _dev(pts, torch.float64, (P, 3), "pts")
        h = ctypes.c_void_p()
        mask = 0
        for pr in (precisions if precisions is not None else (FP64, FP32, BF16X3)):
            mask |= 1 << precision_code(pr)
        check(self._lib.cosim_assemble_component(geom.handle, P, ptr, float(bext_z), mask,
                                                 int(component), _stream(), ctypes.byref(h)))
        self._h = h
        self.component = int(component)
        self.n = geom.n
        self.P = P
        self.device = pts.device
        self.bext_z = float(bext_z)
        # counts the calls that use the plan's workspace (and so end the
        # factor record of the last solve): a record made at generation g is
        # intact while the count is still g
        self._gen = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.cosim_plan_destroy(h)
            self._h = None

    # -- operators ------------------------------------------------------------
    def set_drive(self, loops, power=1.0, phase=0.0, z0: float = 50.0) -> None:
        """Driven ports in series with `loops` (cosim_plan_set_drive): each sends
        sqrt(z0 power) exp(j phase) (Eq. 4; scalars broadcast); [] removes them."""
        loops = np.ascontiguousarray(np.atleast_1d(np.asarray(loops, dtype=np.int32)))
        k = loops.shape[0]
        pw = np.ascontiguousarray(np.broadcast_to(np.asarray(power, dtype=np.float64), (k,)))
        ph = np.ascontiguousarray(np.broadcast_to(np.asarray(phase, dtype=np.float64), (k,)))
        check(self._lib.cosim_plan_set_drive(self._h, k, _host(loops), _host(pw), _host(ph),
                                             float(z0), _stream()))
        self._gen += 1

    def set_refinement(self, enable: bool = True, max_iter: int = 8, tol: float = 0.0) -> None:
        """FP32 factorisation with FP64 refinement above 64 loops
        (cosim_plan_set_refinement); tol 0 chooses it per precision."""
        check(self._lib.cosim_plan_set_refinement(self._h, int(bool(enable)), int(max_iter),
                                                  float(tol)))
        self._gen += 1

    def reserve(self, max_batch: int, max_freq: int) -> None:
        check(self._lib.cosim_plan_reserve(self._h, int(max_batch), int(max_freq)))
        self._gen += 1

    def G(self) -> torch.Tensor:
        out = torch.empty((self.P, self.n), dtype=torch.float64, device=self.device)
        check(self._lib.cosim_plan_copy_G(self._h, ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def M(self) -> np.ndarray:
        out = np.empty((self.n, self.n))
        check(self._lib.cosim_plan_copy_M(self._h, _host(out)))
        return out

    def phi(self) -> np.ndarray:
        out = np.empty(self.n)
        check(self._lib.cosim_plan_copy_phi(self._h, _host(out)))
        return out

    # -- tuning of the fused contraction ------------------------------------------
    def variants(self, precision) -> Tuple[int, int]:
        v = ctypes.c_int(); nv = ctypes.c_int()
        check(self._lib.cosim_plan_get_variant(self._h, precision_code(precision), ctypes.byref(v),
                                               ctypes.byref(nv)))
        return v.value, nv.value

    def set_variant(self, precision, variant: int) -> None:
        check(self._lib.cosim_plan_set_variant(self._h, precision_code(precision), int(variant)))

    def autotune(self, C, omega, T, precision=FP32, loss_mode: int = LOSS_MAG, reps: int = 3):
        """Times every fused-kernel variant on these inputs and keeps the fastest.
        Returns (chosen variant, ms per call of each variant)."""
        prec = precision_code(precision)
        B, F = int(C.shape[0]), int(omega.shape[0])
        _, nv = self.variants(prec)
        self._gen += 1
        ms = np.zeros(nv)
        check(self._lib.cosim_plan_autotune(
            self._h, B, F, _dev(C, torch.float64, (B, self.n), "C"),
            _dev(omega, torch.float64, (F,), "omega"), _dev(T, torch.float64, (self.P,), "T"),
            int(loss_mode), prec, int(reps), _stream(), _host(ms)))
        return self.variants(prec)[0], ms

    # -- phase timing (HIP events on the call's stream) ------------------------
    PHASES = ("solve_forward", "fused_contraction", "solve_adjoint", "reduce")

    def timing(self, max_records: int) -> None:
        check(self._lib.cosim_plan_timing(self._h, int(max_records)))
        self._timing_cap = int(max_records)

    def timing_read(self) -> np.ndarray:
        cap = getattr(self, "_timing_cap", 0)
        out = np.zeros((max(cap, 1), len(self.PHASES)))
        nr = ctypes.c_int()
        check(self._lib.cosim_plan_timing_read(self._h, _host(out), cap, ctypes.byref(nr)))
        return out[:nr.value]

    # -- path -----------------------------------------------------------------
    def solve(self, C: torch.Tensor, omega: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
        """Currents I [B][F][n] and status [B][F] (cosim_solve); the plan keeps
        the factor record for field_backward(reuse=True)."""
        B, F = int(C.shape[0]), int(omega.shape[0])
        self._gen += 1
        I = torch.empty((B, F, self.n), dtype=torch.complex128, device=self.device)
        st = torch.empty((B, F), dtype=torch.int32, device=self.device)
        check(self._lib.cosim_solve(self._h, B, F, _dev(C, torch.float64, (B, self.n), "C"),
                                    _dev(omega, torch.float64, (F,), "omega"),
                                    ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(st.data_ptr()),
                                    _stream()))
        return I, st

    def field(self, I: torch.Tensor, precision=FP64, add_incident: bool = False) -> torch.Tensor:
        """B [B][F][P] = G I (+ bext_z with add_incident), complex128 in FP64,
        complex64 otherwise (cosim_field)."""
        prec = precision_code(precision)
        B, F = int(I.shape[0]), int(I.shape[1])
        dt = torch.complex128 if prec == FP64 else torch.complex64
        Bz = torch.empty((B, F, self.P), dtype=dt, device=self.device)
        check(self._lib.cosim_field(self._h, B, F, _dev(I, torch.complex128, (B, F, self.n), "I"),
                                    prec, int(bool(add_incident)), ctypes.c_void_p(Bz.data_ptr()),
                                    _stream()))
        return Bz

    def factorisations(self) -> int:
        """Batches whose Z this plan has factorised (cosim_plan_factorisations)."""
        v = ctypes.c_longlong()
        check(self._lib.cosim_plan_factorisations(self._h, ctypes.byref(v)))
        return v.value

    def record_generation(self) -> int:
        """The current workspace generation (see field_backward)."""
        return self._gen

    def field_backward(self, C, omega, I, gBz, precision=FP64,
                       reuse: bool = False) -> Tuple[torch.Tensor, torch.Tensor]:
        """dL/dC [B][n] and status [B][F] from the upstream gradient gBz
        (cosim_field_backward).  reuse=True replays the factor record of the
        last solve (which must be of these C and omega, with no call that uses
        the workspace since); False factorises again."""
        B, F = int(C.shape[0]), int(omega.shape[0])
        gC = torch.empty((B, self.n), dtype=torch.float64, device=self.device)
        st = torch.empty((B, F), dtype=torch.int32, device=self.device)
        check(self._lib.cosim_field_backward(
            self._h, B, F, _dev(C, torch.float64, (B, self.n), "C"),
            _dev(omega, torch.float64, (F,), "omega"),
            _dev(I, torch.complex128, (B, F, self.n), "I"),
            _dev(gBz, torch.complex128, (B, F, self.P), "gBz"), precision_code(precision),
            int(bool(reuse)), ctypes.c_void_p(gC.data_ptr()), ctypes.c_void_p(st.data_ptr()),
            _stream()))
        if not reuse:
            self._gen += 1
        return gC, st

    def loss_and_grad(self, C: torch.Tensor, omega: torch.Tensor, T: torch.Tensor,
                      loss_mode: int = LOSS_MAG, precision=FP32, grad: bool = True,
                      out: Optional[Tuple[torch.Tensor, torch.Tensor, torch.Tensor]] = None):
        """Per-configuration loss, dL/dC (or None) and per-system status."""
        prec = precision_code(precision)
        B, F = int(C.shape[0]), int(omega.shape[0])
        self._gen += 1
        if out is None:
            loss = torch.empty((B,), dtype=torch.float64, device=self.device)
            g = torch.empty((B, self.n), dtype=torch.float64, device=self.device) if grad else None
            st = torch.empty((B, F), dtype=torch.int32, device=self.device)
        else:
            loss, g, st = out
        gp = ctypes.c_void_p(g.data_ptr()) if g is not None else ctypes.c_void_p()
        check(self._lib.cosim_loss_and_grad(
            self._h, B, F, _dev(C, torch.float64, (B, self.n), "C"),
            _dev(omega, torch.float64, (F,), "omega"), _dev(T, torch.float64, (self.P,), "T"),
            int(loss_mode), prec, _dev(loss, torch.float64, (B,), "loss"), gp,
            _dev(st, torch.int32, (B, F), "status"), _stream()))
        return loss, g, st


    def loss_and_grad_noalloc(self, C: torch.Tensor, omega: torch.Tensor, T: torch.Tensor,
                              out: Tuple[torch.Tensor, Optional[torch.Tensor], torch.Tensor],
                              loss_mode: int = LOSS_MAG, precision=FP32) -> None:
        """cosim_loss_and_grad_noalloc into caller-allocated outputs
        (loss [B], dL/dC [B][n] or None, status [B][F]): the call itself
        allocates no device memory (64 loops or fewer, bounded size)."""
        prec = precision_code(precision)
        B, F = int(C.shape[0]), int(omega.shape[0])
        loss, g, st = out
        gp = (_dev(g, torch.float64, (B, self.n), "grad") if g is not None else ctypes.c_void_p())
        check(self._lib.cosim_loss_and_grad_noalloc(
            self._h, B, F, _dev(C, torch.float64, (B, self.n), "C"),
            _dev(omega, torch.float64, (F,), "omega"), _dev(T, torch.float64, (self.P,), "T"),
            int(loss_mode), prec, _dev(loss, torch.float64, (B,), "loss"), gp,
            _dev(st, torch.int32, (B, F), "status"), _stream()))

    # -- optimisation driver ----------------------------------------------------
    def loss_and_grad_params(self, C: torch.Tensor, omega: torch.Tensor, T: torch.Tensor,
                             loss_mode: int = LOSS_MAG, precision=FP32):
        """cosim_loss_and_grad_params: (loss [B], dL/dC [B][n], dL/dR [B][n],
        dL/dL [B][n] of a series inductance per loop, dL/dw [B][F], status [B][F])."""
        B, F = int(C.shape[0]), int(omega.shape[0])
        self._gen += 1
        dev = self.device
        loss = torch.empty((B,), dtype=torch.float64, device=dev)
        gC = torch.empty((B, self.n), dtype=torch.float64, device=dev)
        gR = torch.empty((B, self.n), dtype=torch.float64, device=dev)
        gL = torch.empty((B, self.n), dtype=torch.float64, device=dev)
        gw = torch.empty((B, F), dtype=torch.float64, device=dev)
        st = torch.empty((B, F), dtype=torch.int32, device=dev)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr())
        check(self._lib.cosim_loss_and_grad_params(
            self._h, B, F, _dev(C, torch.float64, (B, self.n), "C"),
            _dev(omega, torch.float64, (F,), "omega"), _dev(T, torch.float64, (self.P,), "T"),
            int(loss_mode), precision_code(precision), ptr(loss), ptr(gC), ptr(gR), ptr(gL), ptr(gw),
            ptr(st), _stream()))
        return loss, gC, gR, gL, gw, st

    def resonant_capacitance(self, omega: torch.Tensor, coupled: bool = True) -> torch.Tensor:
        """Eq. 13 per frequency and loop [F][n] (cosim_resonant_capacitance)."""
        F = int(omega.shape[0])
        out = torch.empty((F, self.n), dtype=torch.float64, device=self.device)
        check(self._lib.cosim_resonant_capacitance(self._h, F, _dev(omega, torch.float64, (F,), "omega"),
                                                   int(bool(coupled)), ctypes.c_void_p(out.data_ptr()),
                                                   _stream()))
        return out

    def optimize(self, C: torch.Tensor, omega: torch.Tensor, T: torch.Tensor, steps: int,
                 lr: float = 1e-13, betas=(0.9, 0.999), eps: float = 1e-8, precision=FP32,
                 loss_mode: int = LOSS_MAG, graph: bool = False):
        """Adam on C (updated in place) for `steps` steps of cosim_loss_and_grad +
        cosim_adam_step.  With graph=True one step is captured in a HIP graph and
        replayed.  Returns (loss per step [steps][B], status of the last step)."""
        B, F = int(C.shape[0]), int(omega.shape[0])
        self.reserve(B, F)
        loss = torch.empty((B,), dtype=torch.float64, device=self.device)
        g = torch.empty_like(C)
        st = torch.empty((B, F), dtype=torch.int32, device=self.device)
        m = torch.zeros_like(C)
        v = torch.zeros_like(C)
        t = torch.zeros((1,), dtype=torch.int32, device=self.device)
        hist = torch.empty((steps, B), dtype=torch.float64, device=self.device)

        def one_step():
            self.loss_and_grad(C, omega, T, loss_mode=loss_mode, precision=precision,
                               out=(loss, g, st))
            adam_step(C, g, m, v, t, lr=lr, betas=betas, eps=eps)

        if not graph:
            for k in range(steps):
                one_step()
                hist[k].copy_(loss)
            return hist, st
        # warm the variant choice and the workspace on a copy, then capture
        C0, side = C.clone(), torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.loss_and_grad(C0, omega, T, loss_mode=loss_mode, precision=precision,
                               out=(loss, g, st))
        torch.cuda.current_stream().wait_stream(side)
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            one_step()
        for k in range(steps):
            gr.replay()
            hist[k].copy_(loss)
        return hist, st


class ManyCall:
    """One cosim_loss_and_grad_many call over fixed lists of instances, with
    the tensors checked and the pointer arrays built once: run() enqueues the
    call again on the current stream and returns outs, recomputed from the
    current contents of Cs, omegas and Ts (update them in place; the tensors
    themselves must stay the ones given).  For repeated steps over many
    instances this saves the per-call argument checks (about 6 per instance)."""

    def __init__(self, plans, Cs, omegas, Ts, loss_mode: int = LOSS_MAG, precision=FP32,
                 grad: bool = True, outs=None):
        self.lib = load_library()
        k = self.k = len(plans)
        if not (len(Cs) == len(omegas) == len(Ts) == k):
            raise ValueError("plans, Cs, omegas and Ts must have equal lengths")
        self.prec = precision_code(precision)
        self.loss_mode = int(loss_mode)
        self.plans = list(plans)
        Bs = [int(C.shape[0]) for C in Cs]
        Fs = [int(o.shape[0]) for o in omegas]
        if outs is None:
            outs = []
            for pl, B, F in zip(plans, Bs, Fs):
                outs.append((torch.empty((B,), dtype=torch.float64, device=pl.device),
                             torch.empty((B, pl.n), dtype=torch.float64, device=pl.device) if grad else None,
                             torch.empty((B, F), dtype=torch.int32, device=pl.device)))
        self.outs = outs
        self._keep = (list(Cs), list(omegas), list(Ts))  # the arrays point into these
        ptrs = lambda xs: (ctypes.c_void_p * k)(*[ctypes.c_void_p(x) for x in xs])
        self.arr_p = (ctypes.c_void_p * k)(*[pl._h for pl in plans])
        self.arr_B = (ctypes.c_int * k)(*Bs)
        self.arr_F = (ctypes.c_int * k)(*Fs)
        self.c_p = ptrs([_dev(C, torch.float64, (B, pl.n), "C").value for C, B, pl in zip(Cs, Bs, plans)])
        self.o_p = ptrs([_dev(o, torch.float64, (F,), "omega").value for o, F in zip(omegas, Fs)])
        self.t_p = ptrs([_dev(T, torch.float64, (pl.P,), "T").value for T, pl in zip(Ts, plans)])
        self.l_p = ptrs([o[0].data_ptr() for o in outs])
        self.g_p = ptrs([o[1].data_ptr() for o in outs]) if grad else None
        self.s_p = ptrs([o[2].data_ptr() for o in outs])

    def run(self):
        for pl in self.plans:
            pl._gen += 1
        check(self.lib.cosim_loss_and_grad_many(self.k, self.arr_p, self.arr_B, self.arr_F, self.c_p,
                                                self.o_p, self.t_p, self.loss_mode, self.prec,
                                                self.l_p, self.g_p, self.s_p, _stream()))
        return self.outs


def loss_and_grad_many(plans, Cs, omegas, Ts, loss_mode: int = LOSS_MAG, precision=FP32,
                       grad: bool = True, outs=None):
    """cosim_loss_and_grad_many over independent instances (lists of equal
    length).  Returns lists of per-instance (loss, grad or None, status).
    For repeated calls over the same tensors, ManyCall checks them once."""
    return ManyCall(plans, Cs, omegas, Ts, loss_mode, precision, grad, outs).run()


def capture_loss_and_grad_many(plans, Cs, omegas, Ts, loss_mode: int = LOSS_MAG,
                               precision=FP32, grad: bool = True):
    """One loss_and_grad_many call over the instances captured in a HIP graph.
    Each plan's workspace is reserved for its batch and a first call runs
    outside the capture (on a side stream).  Returns (graph, outs): replaying
    the graph recomputes outs from the current contents of Cs, omegas and Ts
    (update them in place); a call of many small launches becomes one launch.
    Under capture, instances of 64 loops or fewer share launches per padded
    size as in an eager call; instances above 64 loops run their own chains."""
    for pl, C, o in zip(plans, Cs, omegas):
        pl.reserve(int(C.shape[0]), int(o.shape[0]))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        outs = loss_and_grad_many(plans, Cs, omegas, Ts, loss_mode, precision, grad)
    torch.cuda.current_stream().wait_stream(side)
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        loss_and_grad_many(plans, Cs, omegas, Ts, loss_mode, precision, grad, outs=outs)
    return gr, outs


def adam_step(C: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
              step: torch.Tensor, lr: float = 1e-13, betas=(0.9, 0.999), eps: float = 1e-8) -> None:
    """One cosim_adam_step on C (in place); m, v, step are the caller's state."""
    lib = load_library()
    shape = tuple(C.shape)
    count = int(C.numel())
    check(lib.cosim_adam_step(count, _dev(C, torch.float64, shape, "C"),
                              _dev(grad, torch.float64, shape, "grad"),
                              _dev(m, torch.float64, shape, "m"), _dev(v, torch.float64, shape, "v"),
                              _dev(step, torch.int32, (1,), "step"), float(lr), float(betas[0]),
                              float(betas[1]), float(eps), _stream()))


def tanh_projection(theta: torch.Tensor, cmin: float, cmax: float, derivative: bool = False):
    """C = cmin + (cmax - cmin)(1 + tanh theta)/2 (and dC/dtheta) (cosim_tanh_projection)."""
    lib = load_library()
    th = theta.contiguous()
    if th.dtype != torch.float64 or th.device.type != "cuda":
        raise TypeError("theta must be a float64 GPU tensor")
    C = torch.empty_like(th)
    dC = torch.empty_like(th) if derivative else None
    check(lib.cosim_tanh_projection(th.numel(), ctypes.c_void_p(th.data_ptr()), float(cmin),
                                    float(cmax), ctypes.c_void_p(C.data_ptr()),
                                    ctypes.c_void_p(dC.data_ptr()) if dC is not None else None,
                                    _stream()))
    return (C, dC) if derivative else C


def clip_(x: torch.Tensor, lo: float, hi: float) -> torch.Tensor:
    """Clamp x to [lo, hi] in place (cosim_clip)."""
    lib = load_library()
    if x.dtype != torch.float64 or x.device.type != "cuda" or not x.is_contiguous():
        raise TypeError("x must be a contiguous float64 GPU tensor")
    check(lib.cosim_clip(x.numel(), ctypes.c_void_p(x.data_ptr()), float(lo), float(hi), _stream()))
    return x


class CosimField(torch.autograd.Function):
    """B_z = f(C) with the library's hand-written adjoint as backward.

    forward: cosim_solve (which keeps the factor record in the plan) +
    cosim_field on the matrix cores in `precision`, plus the incident field
    with add_incident; backward: cosim_field_backward in the same precision,
    replaying the forward factorisation (Z is complex symmetric, so it serves
    Z^T) when no other call has used the plan's workspace since the forward,
    else factorising again; it returns the real dL/dC."""

    @staticmethod
    def forward(ctx, C, plan: Plan, omega, precision=FP64, add_incident=False):
        Cd = C.detach().contiguous()
        I, _ = plan.solve(Cd, omega)
        ctx.gen = plan.record_generation()
        Bz = plan.field(I, precision, add_incident)
        ctx.plan = plan
        ctx.precision = precision
        ctx.save_for_backward(Cd, omega, I)
        return Bz

    @staticmethod
    def backward(ctx, gBz):
        C, omega, I = ctx.saved_tensors
        g = gBz.to(torch.complex128).contiguous()
        reuse = ctx.plan.record_generation() == ctx.gen
        gC, _ = ctx.plan.field_backward(C, omega, I, g, ctx.precision, reuse=reuse)
        return gC, None, None, None, None


def cosim_field(C: torch.Tensor, plan: Plan, omega: torch.Tensor, precision=FP64,
                add_incident: bool = False) -> torch.Tensor:
    return CosimField.apply(C, plan, omega, precision_code(precision), bool(add_incident))


# ---------------------------------------------------------------------------
# S-parameter pipeline (include/cosim_sparam.h)
# ---------------------------------------------------------------------------

class SParamPlan:
    """Exports of an n0-port structure (S0 [F][n0][n0] and per-port fields
    [F][P][ncomp][n0], complex128 on the GPU) connected through
    S_C = S_C,const + S_C,var (variable entries at rows idx_x, columns idx_y) to
    n1 external ports driven by the waves `exc` (cosim_sp_create)."""

    def __init__(self, S0: torch.Tensor, fields: torch.Tensor, idx_x, idx_y, exc,
                 sc_const: Optional[torch.Tensor] = None, precisions=("fp64", "fp32")):
        self._lib = load_library()
        F, n0 = int(S0.shape[0]), int(S0.shape[1])
        P, ncomp = int(fields.shape[1]), int(fields.shape[2])
        self.idx_x = np.ascontiguousarray(idx_x, dtype=np.int32)
        self.idx_y = np.ascontiguousarray(idx_y, dtype=np.int32)
        self.exc = np.ascontiguousarray(np.atleast_1d(exc), dtype=np.complex128)
        n1 = int(self.exc.shape[0])
        nvar = int(self.idx_x.shape[0])
        if self.idx_y.shape[0] != nvar:
            raise ValueError("idx_x and idx_y differ in length")
        N = n0 + n1
        s0 = _dev(S0, torch.complex128, (F, n0, n0), "S0")
        fp = _dev(fields, torch.complex128, (F, P, ncomp, n0), "fields")
        scp = None if sc_const is None else _dev(sc_const, torch.complex128, (F, N, N), "sc_const")
        mask = 0
        for pr in precisions:
            mask |= 1 << precision_code(pr)
        h = ctypes.c_void_p()
        check(self._lib.cosim_sp_create(n0, n1, F, P, ncomp, s0, fp, scp, nvar,
                                        _host(self.idx_x) if nvar else None,
                                        _host(self.idx_y) if nvar else None, _host(self.exc),
                                        mask, _stream(), ctypes.byref(h)))
        self._h = h
        self.n0, self.n1, self.F, self.P, self.ncomp, self.nvar = n0, n1, F, P, ncomp, nvar
        self.device = S0.device

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.cosim_sp_destroy(h)
            self._h = None

    def reserve(self, max_batch: int) -> None:
        check(self._lib.cosim_sp_reserve(self._h, int(max_batch)))

    def _values(self, values: torch.Tensor, B: int):
        if self.nvar == 0:
            return None
        return _dev(values, torch.complex128, (B, self.F, self.nvar), "values")

    def field(self, values: torch.Tensor, want_field: bool = True):
        """Returns (x [B][F][n0], B_comb [B][F][P][ncomp] or None, status [B][F])."""
        B = int(values.shape[0])
        x = torch.empty((B, self.F, self.n0), dtype=torch.complex128, device=self.device)
        Bc = (torch.empty((B, self.F, self.P, self.ncomp), dtype=torch.complex128, device=self.device)
              if want_field else None)
        st = torch.empty((B, self.F), dtype=torch.int32, device=self.device)
        check(self._lib.cosim_sp_field(self._h, B, self._values(values, B),
                                       ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(Bc.data_ptr()) if Bc is not None else None,
                                       ctypes.c_void_p(st.data_ptr()), _stream()))
        return x, Bc, st

    def loss_and_grad(self, values: torch.Tensor, T: torch.Tensor, comp: int = 0,
                      loss_mode: int = LOSS_MAG, precision=FP64, grad: bool = True, out=None):
        """Returns (loss [B], 2 dL/dconj(values) [B][F][nvar] or None, status [B][F])."""
        B = int(values.shape[0])
        if out is None:
            loss = torch.empty((B,), dtype=torch.float64, device=self.device)
            g = (torch.empty((B, self.F, self.nvar), dtype=torch.complex128, device=self.device)
                 if grad else None)
            st = torch.empty((B, self.F), dtype=torch.int32, device=self.device)
        else:
            loss, g, st = out
        check(self._lib.cosim_sp_loss_and_grad(
            self._h, B, self._values(values, B), _dev(T, torch.float64, (self.P,), "T"), int(comp),
            int(loss_mode), precision_code(precision), ctypes.c_void_p(loss.data_ptr()),
            ctypes.c_void_p(g.data_ptr()) if g is not None else None,
            ctypes.c_void_p(st.data_ptr()), _stream()))
        return loss, g, st


def sp_rc(R: torch.Tensor, C: torch.Tensor, omega: torch.Tensor, z0: float = 50.0,
          out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Reflection of the RC loads (Eq. 2-3) [B][F][n], or into the first n
    columns of out [B][F][ld] (cosim_sp_rc)."""
    lib = load_library()
    B, n = int(C.shape[0]), int(C.shape[1])
    F = int(omega.shape[0])
    if out is None:
        out = torch.empty((B, F, n), dtype=torch.complex128, device=C.device)
    ld = int(out.shape[2])
    check(lib.cosim_sp_rc(B, F, n, _dev(R, torch.float64, (n,), "R"), _dev(C, torch.float64, (B, n), "C"),
                          _dev(omega, torch.float64, (F,), "omega"), float(z0),
                          _dev(out, torch.complex128, (B, F, ld), "out"), ld, _stream()))
    return out


def sp_rc_backward(R: torch.Tensor, C: torch.Tensor, omega: torch.Tensor, g: torch.Tensor,
                   z0: float = 50.0) -> torch.Tensor:
    """dL/dC [B][n] from g = 2 dL/dconj(Gamma) in the first n columns of g
    [B][F][ld] (cosim_sp_rc_backward)."""
    lib = load_library()
    B, n = int(C.shape[0]), int(C.shape[1])
    F = int(omega.shape[0])
    ld = int(g.shape[2])
    gC = torch.empty((B, n), dtype=torch.float64, device=C.device)
    check(lib.cosim_sp_rc_backward(B, F, n, _dev(R, torch.float64, (n,), "R"),
                                   _dev(C, torch.float64, (B, n), "C"),
                                   _dev(omega, torch.float64, (F,), "omega"), float(z0),
                                   _dev(g, torch.complex128, (B, F, ld), "g"), ld,
                                   ctypes.c_void_p(gC.data_ptr()), _stream()))
    return gC
