"""Python binding of the MI355X LKS library (``liblks.so``, C ABI in include/lks.h).

Argument marshalling only: every stage of the forward march, the adjoint and
the sensitivities runs in the library's HIP kernels.  PyTorch provides device
memory (including the workspace) and the current stream.  If the library has
not been built this module raises on first use; there is no fallback.

States use the library layout: [d+1][N] of the state dtype, plane 0 holds
p - 1/3, planes 1..d the velocity.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

from .srcdigest import source_digest

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblks.so")

LKS_OK, LKS_EINVAL, LKS_EDOMAIN, LKS_EUNSTABLE, LKS_EHIP = range(5)
_NAMES = {0: "LKS_OK", 1: "LKS_EINVAL", 2: "LKS_EDOMAIN", 3: "LKS_EUNSTABLE", 4: "LKS_EHIP"}


class LksError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_NAMES.get(status, status)}: {message}")
        self.status = status


class LksProblem(C.Structure):
    _fields_ = [
        ("d", C.c_int32), ("precision", C.c_int32), ("n", C.c_int32 * 3), ("bc", C.c_int32 * 3),
        ("u_wall", C.c_double * 18), ("nu", C.c_double), ("kappa_max", C.c_double),
        ("q", C.c_double), ("m", C.c_int32 * 3), ("margin", C.c_int32),
        ("xg_min", C.c_double * 3), ("xg_max", C.c_double * 3), ("th_min", C.c_double),
        ("th_max", C.c_double), ("nt", C.c_int32), ("r_t", C.c_int32), ("r_w", C.c_int32),
        ("tgt_lo", C.c_int32 * 3), ("tgt_hi", C.c_int32 * 3), ("ndir", C.c_double * 3),
        ("phi", C.c_double), ("ckpt_k", C.c_int32), ("body_tape", C.c_int32),
        ("scheme", C.c_int32), ("objective", C.c_int32), ("w_d", C.c_double),
        ("w_t", C.c_double), ("l_m", C.c_double), ("rot", C.c_int32),
        ("tilt_min", C.c_double * 2), ("tilt_max", C.c_double * 2),
    ]


class LksOptState(C.Structure):
    _fields_ = [
        ("level", C.c_int32), ("iter", C.c_int32), ("total", C.c_int32), ("beta", C.c_double),
        ("J", C.c_double), ("G", C.c_double * 3), ("gamma", C.c_void_p), ("chi", C.c_void_p),
        ("psi", C.c_void_p), ("dJ_dgamma", C.c_void_p), ("dJ_dchi", C.c_void_p),
        ("dJ_dpsi", C.c_void_p), ("dG1_dgamma", C.c_void_p), ("dG2_dgamma", C.c_void_p),
        ("dG3_dpsi", C.c_void_p),
    ]


class LksOptOptions(C.Structure):
    _fields_ = [
        ("n_cont", C.c_int32), ("beta", C.POINTER(C.c_double)), ("n_opt", C.c_int32),
        ("radius", C.c_double), ("eta", C.c_double), ("tol", C.c_double), ("vmax", C.c_double),
        ("omega_max", C.c_double), ("p_omega", C.c_double), ("g_active", C.c_int32),
        ("periodic", C.c_int32),
    ]


class LksOptResult(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("levels", C.c_int32), ("stopped", C.c_int32),
                ("J_last", C.c_double)]


UPDATE_FN = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.POINTER(LksOptState), C.c_void_p)

_lib = None
_VP = C.c_void_p


def lib():
    """Load liblks.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.lks_last_error.restype = C.c_char_p
        L.lks_source_digest.restype = C.c_char_p
        want = source_digest()
        have = L.lks_source_digest().decode()
        if want is not None and have != want:
            raise RuntimeError(f"{LIB_PATH} was built from other sources (digest {have[:12]}, "
                               f"sources {want[:12]}): rebuild it with __graft_entry__.build()")
        L.lks_plan_create.argtypes = [C.POINTER(LksProblem), C.POINTER(_VP), C.POINTER(C.c_size_t)]
        L.lks_plan_destroy.argtypes = [_VP]
        L.lks_plan_set_graphs.argtypes = [_VP, C.c_int32]
        L.lks_plan_set_zseg.argtypes = [_VP, C.c_int32]
        L.lks_forward.argtypes = [_VP] * 9
        L.lks_adjoint.argtypes = [_VP] * 12
        L.lks_map_design_to_grid.argtypes = [_VP] * 7
        L.lks_sensitivities.argtypes = [_VP] * 7
        L.lks_motion.argtypes = [_VP] * 5
        L.lks_kappa_ref.argtypes = [_VP] * 4
        L.lks_step.argtypes = [_VP] * 6
        L.lks_step_adjoint.argtypes = [_VP] * 10
        L.lks_map_adjoint.argtypes = [_VP] * 8
        L.lks_map_adjoint_blocks.argtypes = [_VP]
        L.lks_map_adjoint_blocks.restype = C.c_int32
        L.lks_profile_enable.argtypes = [C.c_int32]
        L.lks_profile_read.argtypes = [C.POINTER(C.c_char_p), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int64), C.c_int32]
        L.lks_profile_read.restype = C.c_int32
        L.lks_batch_run.argtypes = [C.c_int32] + [_VP] * 11
        D = C.c_double
        L.lks_design_filter.argtypes = [_VP, _VP, D, D, D, _VP, _VP]
        L.lks_design_filter_adjoint.argtypes = [_VP, _VP, D, D, D, _VP, _VP, _VP, _VP]
        L.lks_design_filter_adjoint_noalloc.argtypes = [_VP, _VP, D, D, D, _VP, _VP, _VP]
        L.lks_optimize_scratch_bytes.argtypes = [_VP]
        L.lks_optimize_scratch_bytes.restype = C.c_size_t
        L.lks_optimize.argtypes = [_VP, _VP, C.POINTER(LksOptOptions), _VP, _VP, _VP, _VP,
                                   UPDATE_FN, _VP, _VP, C.POINTER(LksOptResult), _VP]
        L.lks_constraints.argtypes = [_VP] * 5 + [D, D, D] + [_VP] * 5
        _lib = L
    return _lib


def _check(status: int):
    if status != LKS_OK:
        raise LksError(status, lib().lks_last_error().decode(errors="replace"))


def to_struct(p) -> LksProblem:
    s = LksProblem()
    s.d = p.d
    s.precision = p.precision
    for a in range(3):
        s.n[a] = p.n[a] if a < p.d else 1
        s.bc[a] = p.bc[a] if a < p.d else 0
        s.m[a] = p.m[a] if a < p.d else 1
        s.xg_min[a] = p.xg_min[a]
        s.xg_max[a] = p.xg_max[a]
        s.tgt_lo[a] = p.tgt_lo[a]
        s.tgt_hi[a] = p.tgt_hi[a]
        s.ndir[a] = p.ndir[a]
    flat = [float(v) for ax in p.u_wall for side in ax for v in side]
    for k in range(18):
        s.u_wall[k] = flat[k]
    s.nu, s.kappa_max, s.q = p.nu, p.kappa_max, p.q
    s.margin = p.margin
    s.th_min, s.th_max = p.th_min, p.th_max
    s.nt, s.r_t, s.r_w = p.nt, p.r_t, p.r_w
    s.phi = p.phi
    s.ckpt_k = p.ckpt_k
    s.body_tape = p.body_tape
    s.scheme = p.scheme
    s.objective = p.objective
    s.w_d, s.w_t, s.l_m = p.w_d, p.w_t, p.l_m
    s.rot = getattr(p, "rot", 0)
    for k in range(2):
        s.tilt_min[k] = p.tilt_min[k]
        s.tilt_max[k] = p.tilt_max[k]
    return s


def motion_width(p) -> int:
    """Values per motion row: 8, or 12 with three rotation angles."""
    return 12 if getattr(p, "rot", 0) == 1 else 8


def psi_per_step(p) -> int:
    """Rotation design variables per step: 1, or 3 with three angles."""
    return 3 if getattr(p, "rot", 0) == 1 else 1


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


class Plan:
    """A validated problem plus its device workspace (allocated by torch)."""

    def __init__(self, problem, device: str = "cuda"):
        self.problem = problem
        self.device = torch.device(device)
        self._s = to_struct(problem)
        h = _VP()
        nbytes = C.c_size_t()
        _check(lib().lks_plan_create(C.byref(self._s), C.byref(h), C.byref(nbytes)))
        self.handle = h
        self.workspace_bytes = nbytes.value
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        self.dtype = torch.float32 if problem.precision == 0 else torch.float64
        # forward marches run on this plan's workspace so far; the adjoint
        # reverses the last one only
        self.generation = 0

    def set_graphs(self, on: bool):
        """Replay the time loops from captured hipGraphs (default) or launch eagerly."""
        _check(lib().lks_plan_set_graphs(self.handle, 1 if on else 0))

    def set_zseg(self, zseg: int):
        """3D step kernels: z planes per block segment (0 = automatic)."""
        _check(lib().lks_plan_set_zseg(self.handle, int(zseg)))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.lks_plan_destroy(h)

    # ----------------------------------------------------------- helpers
    def _f64(self, a) -> torch.Tensor:
        return torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()

    def _st(self, a) -> torch.Tensor:
        return torch.as_tensor(a, dtype=self.dtype, device=self.device).contiguous()

    @property
    def adj_state_size(self) -> int:
        """Values of adj_terminal / adj_initial: the state's with the exact
        adjoint; with the ALKS also its carried state p~, u~ and the
        symmetric s~ ([(d+1) + 1 + d + d(d+1)/2][N])."""
        p = self.problem
        if p.scheme == 1:
            return (p.d + 1 + 1 + p.d + p.d * (p.d + 1) // 2) * p.N
        return self.state_size

    @property
    def state_size(self) -> int:
        p = self.problem
        return (p.d + 1) * p.N

    # -------------------------------------------------------- full path
    def forward(self, gamma, chi, psi, state0=None, want_final: bool = False):
        """Forward march; returns (J3 device tensor [J, E, V], final state or None)."""
        g, c, s = self._f64(gamma), self._f64(chi), self._f64(psi)
        st0 = None if state0 is None else self._st(state0)
        fin = torch.empty(self.state_size, dtype=self.dtype, device=self.device) if want_final else None
        J3 = torch.empty(3, dtype=torch.float64, device=self.device)
        self._keep = (g, c, s)
        self.generation += 1
        _check(lib().lks_forward(self.handle, _ptr(g), _ptr(c), _ptr(s), _ptr(st0), _ptr(fin),
                                 _ptr(self.workspace), _ptr(J3), _stream()))
        return J3, fin

    def adjoint(self, gamma, chi, psi, dJ=None, adj_terminal=None, want_initial: bool = False):
        """Discrete adjoint of the preceding forward; returns gradients."""
        p = self.problem
        g, c, s = self._f64(gamma), self._f64(chi), self._f64(psi)
        seed = self._f64([1.0]) if dJ is None else self._f64(dJ).reshape(1)
        at = None if adj_terminal is None else self._st(adj_terminal)
        if at is not None and at.numel() != self.adj_state_size:
            raise ValueError(f"adj_terminal needs {self.adj_state_size} values")
        ai = (torch.empty(self.adj_state_size, dtype=self.dtype, device=self.device)
              if want_initial else None)
        dg = torch.empty(p.M, dtype=torch.float64, device=self.device)
        dc = torch.empty(p.nt * 3, dtype=torch.float64, device=self.device)
        dp = torch.empty(p.nt * psi_per_step(p), dtype=torch.float64, device=self.device)
        _check(lib().lks_adjoint(self.handle, _ptr(g), _ptr(c), _ptr(s), _ptr(self.workspace),
                                 _ptr(seed), _ptr(at), _ptr(ai), _ptr(dg), _ptr(dc), _ptr(dp),
                                 _stream()))
        return {"dgamma": dg, "dchi": dc.reshape(p.nt, 3), "dpsi": self._psi_view(dp),
                "adj_initial": ai}

    def _psi_view(self, t):
        return t.reshape(self.problem.nt, 3) if psi_per_step(self.problem) == 3 else t

    def sensitivities(self, gamma):
        p = self.problem
        g = self._f64(gamma)
        dg = torch.empty(p.M, dtype=torch.float64, device=self.device)
        dc = torch.empty(p.nt * 3, dtype=torch.float64, device=self.device)
        dp = torch.empty(p.nt * psi_per_step(p), dtype=torch.float64, device=self.device)
        _check(lib().lks_sensitivities(self.handle, _ptr(g), _ptr(self.workspace), _ptr(dg),
                                       _ptr(dc), _ptr(dp), _stream()))
        return dg, dc.reshape(p.nt, 3), self._psi_view(dp)

    # ---------------------------------------------------- optimiser side
    def design_filter(self, gamma, radius: float, beta: float, eta: float):
        """Density filter and Heaviside projection (Sec. 3.1): gamma -> the
        projected density that forward() takes."""
        g = self._f64(gamma)
        out = torch.empty(self.problem.M, dtype=torch.float64, device=self.device)
        _check(lib().lks_design_filter(self.handle, _ptr(g), C.c_double(radius), C.c_double(beta),
                                       C.c_double(eta), _ptr(out), _stream()))
        return out

    def design_filter_adjoint(self, gamma, radius: float, beta: float, eta: float, dJ_dphys):
        """Chain rule of design_filter: dJ/d(projected density) -> dJ/dgamma."""
        g, gb = self._f64(gamma), self._f64(dJ_dphys)
        work = torch.empty(self.problem.M, dtype=torch.float64, device=self.device)
        out = torch.empty(self.problem.M, dtype=torch.float64, device=self.device)
        _check(lib().lks_design_filter_adjoint(self.handle, _ptr(g), C.c_double(radius),
                                               C.c_double(beta), C.c_double(eta), _ptr(gb),
                                               _ptr(work), _ptr(out), _stream()))
        return out

    def design_filter_adjoint_noalloc(self, gamma, radius: float, beta: float, eta: float,
                                      dJ_dphys, out=None):
        """design_filter_adjoint with the library's fixed device scratch
        (lks_design_filter_adjoint_noalloc); `out` (M doubles) may be given."""
        g, gb = self._f64(gamma), self._f64(dJ_dphys)
        if out is None:
            out = torch.empty(self.problem.M, dtype=torch.float64, device=self.device)
        _check(lib().lks_design_filter_adjoint_noalloc(self.handle, _ptr(g), C.c_double(radius),
                                                       C.c_double(beta), C.c_double(eta),
                                                       _ptr(gb), _ptr(out), _stream()))
        return out

    def constraints(self, gamma_phys, chi, psi, vmax: float, omega_max: float, p_omega: float):
        """(G1, G2, G3) of Sec. 2.6 and dG1, dG2 (w.r.t. the projected
        density) and dG3/dpsi."""
        p = self.problem
        g, c, s = self._f64(gamma_phys), self._f64(chi), self._f64(psi)
        G = torch.empty(3, dtype=torch.float64, device=self.device)
        d1 = torch.empty(p.M, dtype=torch.float64, device=self.device)
        d2 = torch.empty(p.M, dtype=torch.float64, device=self.device)
        d3 = torch.empty(p.nt * psi_per_step(p), dtype=torch.float64, device=self.device)
        _check(lib().lks_constraints(self.handle, _ptr(self.workspace), _ptr(g), _ptr(c), _ptr(s),
                                     C.c_double(vmax), C.c_double(omega_max), C.c_double(p_omega),
                                     _ptr(G), _ptr(d1), _ptr(d2), _ptr(d3), _stream()))
        return G, d1, d2, d3

    # ---------------------------------------------------- single stages
    def motion(self, chi, psi):
        c, s = self._f64(chi), self._f64(psi)
        W = motion_width(self.problem)
        out = torch.empty(self.problem.nt * W, dtype=torch.float64, device=self.device)
        _check(lib().lks_motion(self.handle, _ptr(c), _ptr(s), _ptr(out), _stream()))
        return out.reshape(self.problem.nt, W)

    def kappa_ref(self, gamma):
        g = self._f64(gamma)
        out = torch.empty(self.problem.Mtot, dtype=self.dtype, device=self.device)
        _check(lib().lks_kappa_ref(self.handle, _ptr(g), _ptr(out), _stream()))
        return out

    def map(self, kref, motion8):
        p = self.problem
        kr, m = self._st(kref), self._f64(motion8)
        k = torch.empty(p.N, dtype=self.dtype, device=self.device)
        us = torch.empty(p.d * p.N, dtype=self.dtype, device=self.device)
        _check(lib().lks_map_design_to_grid(self.handle, _ptr(kr), _ptr(m), _ptr(k), _ptr(us),
                                            _ptr(self.workspace), _stream()))
        return k, us

    def step(self, state, kappa, us):
        si, k, u = self._st(state), self._st(kappa), self._st(us)
        out = torch.empty_like(si)
        _check(lib().lks_step(self.handle, _ptr(si), _ptr(k), _ptr(u), _ptr(out), _stream()))
        return out

    def step_adjoint(self, state_in, state_out, kappa, us, lam):
        p = self.problem
        si, so, k, u, l = (self._st(v) for v in (state_in, state_out, kappa, us, lam))
        lp = torch.empty_like(si)
        kb = torch.empty(p.N, dtype=self.dtype, device=self.device)
        ub = torch.empty(p.d * p.N, dtype=self.dtype, device=self.device)
        _check(lib().lks_step_adjoint(self.handle, _ptr(si), _ptr(so), _ptr(k), _ptr(u), _ptr(l),
                                      _ptr(lp), _ptr(kb), _ptr(ub), _stream()))
        return lp, kb, ub

    def map_adjoint(self, kref, motion8, kbar, usbar):
        p = self.problem
        kr, m, kb, ub = self._st(kref), self._f64(motion8), self._st(kbar), self._st(usbar)
        nblk = lib().lks_map_adjoint_blocks(self.handle)
        out = torch.empty(p.Mtot, dtype=torch.float64, device=self.device)
        W = motion_width(p)
        mb = torch.empty(W * (nblk + 1), dtype=torch.float64, device=self.device)
        _check(lib().lks_map_adjoint(self.handle, _ptr(kr), _ptr(m), _ptr(kb), _ptr(ub), _ptr(out),
                                     _ptr(mb), _stream()))
        return out, mb[:W].clone()


def optimize(plan: "Plan", gamma, chi, psi, update, *, beta=(1.0,), n_opt: int = 100,
             radius: float = 4.8, eta: float = 0.5, tol: float = 1e-6, vmax: float = 1.0,
             omega_max: float = 1.0, p_omega: float = 16.0, g_active: int = 0,
             periodic: bool = True):
    """Algorithm 1 (lks_optimize): continuation over `beta`, up to n_opt
    iterations per level, with the caller's optimiser step
    update(state) -> bool (True stops), where state is a dict of device
    tensors (gamma, chi, psi to update in place; dJ_dgamma, dJ_dchi, dJ_dpsi,
    dG1_dgamma, dG2_dgamma, dG3_dpsi) and the scalars level, iter, total,
    beta, J, G.  Returns (gamma, chi, psi, history [iterations][4],
    result dict)."""
    p = plan.problem
    g = plan._f64(gamma).clone().reshape(-1)
    c = plan._f64(chi).clone().reshape(-1)
    s = plan._f64(psi).clone().reshape(-1)
    L = lib()
    scratch = torch.empty(L.lks_optimize_scratch_bytes(plan.handle), dtype=torch.uint8,
                          device=plan.device)
    base = scratch.data_ptr()
    f64 = scratch.view(torch.float64)
    nps = psi_per_step(p)
    sizes = {"dJ_dgamma": p.M, "dJ_dchi": 3 * p.nt, "dJ_dpsi": nps * p.nt,
             "dG1_dgamma": p.M, "dG2_dgamma": p.M, "dG3_dpsi": nps * p.nt}
    own = {g.data_ptr(): g, c.data_ptr(): c, s.data_ptr(): s}

    def view(ptr, n):
        if ptr in own:
            return own[ptr]
        off = ptr - base
        assert off >= 0 and off % 8 == 0 and off // 8 + n <= f64.numel()
        return f64[off // 8: off // 8 + n]

    def cb(_user, stp, _stream):
        st = stp.contents
        d = {"level": st.level, "iter": st.iter, "total": st.total, "beta": st.beta, "J": st.J,
             "G": tuple(st.G), "gamma": view(st.gamma, p.M), "chi": view(st.chi, 3 * p.nt),
             "psi": view(st.psi, nps * p.nt)}
        for k, n in sizes.items():
            d[k] = view(getattr(st, k), n)
        try:
            return 1 if update(d) else 0
        except Exception:  # an exception in the step stops the loop
            import traceback
            traceback.print_exc()
            return 1

    fn = UPDATE_FN(cb)
    betas = (C.c_double * len(beta))(*beta)
    opt = LksOptOptions(len(beta), betas, n_opt, radius, eta, tol, vmax, omega_max, p_omega,
                        g_active, 1 if periodic else 0)
    hist = (C.c_double * (4 * len(beta) * n_opt))()
    res = LksOptResult()
    _check(L.lks_optimize(plan.handle, _ptr(plan.workspace), C.byref(opt), _ptr(g), _ptr(c),
                          _ptr(s), _ptr(scratch), fn, None, hist, C.byref(res), _stream()))
    plan.generation += res.iterations
    history = [tuple(hist[4 * i: 4 * i + 4]) for i in range(res.iterations)]
    out = {"iterations": res.iterations, "levels": res.levels, "stopped": res.stopped,
           "J_last": res.J_last}
    return g, c.reshape(p.nt, 3), plan._psi_view(s), history, out


class LKSObjective(torch.autograd.Function):
    """J1(gamma, chi, psi) with the hand-written discrete adjoint as backward.

    forward runs the checkpointed forward march (lks_forward); backward runs
    lks_adjoint, which recomputes each K-step segment from its checkpoint."""

    @staticmethod
    def forward(ctx, gamma, chi, psi, plan: Plan):
        J3, _ = plan.forward(gamma, chi, psi)
        ctx.plan = plan
        ctx.generation = plan.generation
        ctx.save_for_backward(gamma, chi, psi)
        return J3[0].clone()

    @staticmethod
    def backward(ctx, gJ):
        gamma, chi, psi = ctx.saved_tensors
        plan = ctx.plan
        if plan.generation != ctx.generation:
            # another march has run on the plan since this one (a second
            # apply, or a direct forward): march again for these inputs, so
            # the adjoint reverses the right one
            plan.forward(gamma, chi, psi)
        g = plan.adjoint(gamma, chi, psi, dJ=gJ.detach().reshape(1).to(torch.float64))
        p = plan.problem
        return (g["dgamma"].reshape(gamma.shape).to(gamma.dtype),
                g["dchi"].reshape(chi.shape).to(chi.dtype),
                g["dpsi"].reshape(psi.shape).to(psi.dtype), None)


class Batch:
    """Independent instances run as one captured graph (lks_batch_run).

    Inputs are copied into buffers owned by this object, so repeated calls
    keep the same pointer tables and replay the captured graph."""

    def __init__(self, plans):
        self.plans = list(plans)
        n = len(self.plans)
        dev = self.plans[0].device
        f64 = dict(dtype=torch.float64, device=dev)
        self.g = [torch.empty(pl.problem.M, **f64) for pl in self.plans]
        self.c = [torch.empty(pl.problem.nt * 3, **f64) for pl in self.plans]
        self.s = [torch.empty(pl.problem.nt * psi_per_step(pl.problem), **f64)
                   for pl in self.plans]
        self.J = [torch.empty(3, **f64) for _ in self.plans]
        self.dg = [torch.empty(pl.problem.M, **f64) for pl in self.plans]
        self.dc = [torch.empty(pl.problem.nt * 3, **f64) for pl in self.plans]
        self.dp = [torch.empty(pl.problem.nt * psi_per_step(pl.problem), **f64)
                   for pl in self.plans]
        self.seed = torch.ones(n, **f64)
        tab = lambda ts: (_VP * n)(*[t.data_ptr() for t in ts])
        self._tabs = dict(plans=(_VP * n)(*[pl.handle.value for pl in self.plans]),
                          g=tab(self.g), c=tab(self.c), s=tab(self.s),
                          ws=tab([pl.workspace for pl in self.plans]), J=tab(self.J),
                          dg=tab(self.dg), dc=tab(self.dc), dp=tab(self.dp))

    def run(self, gammas, chis, psis, dJ=None):
        """Returns a list of (J3, {"dgamma", "dchi", "dpsi"}) device tensors."""
        for k, pl in enumerate(self.plans):
            self.g[k].copy_(torch.as_tensor(gammas[k], dtype=torch.float64).reshape(-1))
            self.c[k].copy_(torch.as_tensor(chis[k], dtype=torch.float64).reshape(-1))
            self.s[k].copy_(torch.as_tensor(psis[k], dtype=torch.float64).reshape(-1))
        if dJ is not None:
            self.seed.copy_(torch.as_tensor(dJ, dtype=torch.float64).reshape(-1))
        t = self._tabs
        _check(lib().lks_batch_run(len(self.plans), t["plans"], t["g"], t["c"], t["s"], t["ws"],
                                   t["J"], _ptr(self.seed), t["dg"], t["dc"], t["dp"],
                                   _stream()))
        for pl in self.plans:
            pl._keep = None
            pl.generation += 1
        return [(self.J[k], {"dgamma": self.dg[k],
                             "dchi": self.dc[k].reshape(pl.problem.nt, 3),
                             "dpsi": pl._psi_view(self.dp[k])})
                for k, pl in enumerate(self.plans)]


def profile_enable(on: bool = True):
    _check(lib().lks_profile_enable(1 if on else 0))


def profile_read(cap: int = 32):
    names = (C.c_char_p * cap)()
    tot = (C.c_double * cap)()
    cnt = (C.c_int64 * cap)()
    k = lib().lks_profile_read(names, tot, cnt, cap)
    return {names[i].decode(): (tot[i], cnt[i]) for i in range(k)}
