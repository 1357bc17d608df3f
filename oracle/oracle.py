"""ctypes wrapper of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this module.  It loads ``liblks_oracle.so`` built from ``lks_oracle.cpp`` in
this directory (``build()`` compiles it with g++ -O2, no fast-math).

Fields are numpy float64 arrays; analysis states are [d+1][N] with plane 0 the
pressure p itself (the GPU library stores p - 1/3 instead; callers convert).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lks_oracle.cpp")
LIB = os.environ.get("ORACLE_LIB_OVERRIDE") or os.path.join(HERE, "liblks_oracle.so")


class OrcProblem(C.Structure):
    _fields_ = [
        ("d", C.c_int32), ("n", C.c_int32 * 3), ("bc", C.c_int32 * 3),
        ("u_wall", C.c_double * 18), ("dp_seam", C.c_double * 3), ("nu", C.c_double),
        ("kappa_max", C.c_double), ("q", C.c_double), ("m", C.c_int32 * 3),
        ("margin", C.c_int32), ("xg_min", C.c_double * 3), ("xg_max", C.c_double * 3),
        ("th_min", C.c_double), ("th_max", C.c_double), ("nt", C.c_int32),
        ("r_t", C.c_int32), ("r_w", C.c_int32), ("tgt_lo", C.c_int32 * 3),
        ("tgt_hi", C.c_int32 * 3), ("ndir", C.c_double * 3), ("phi", C.c_double),
        ("objective", C.c_int32), ("w_d", C.c_double), ("w_t", C.c_double), ("l_m", C.c_double),
        ("rot", C.c_int32), ("tilt_min", C.c_double * 2), ("tilt_max", C.c_double * 2),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle shared library (plain g++ -O2)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
    return _lib


def to_struct(p) -> OrcProblem:
    s = OrcProblem()
    s.d = p.d
    for a in range(3):
        s.n[a] = p.n[a] if a < p.d else 1
        s.bc[a] = p.bc[a]
        s.dp_seam[a] = p.dp_seam[a]
        s.m[a] = p.m[a] if a < p.d else 1
        s.xg_min[a] = p.xg_min[a]
        s.xg_max[a] = p.xg_max[a]
        s.tgt_lo[a] = p.tgt_lo[a]
        s.tgt_hi[a] = p.tgt_hi[a]
        s.ndir[a] = p.ndir[a]
    uw = np.asarray(p.u_wall, dtype=np.float64).reshape(18)
    for k in range(18):
        s.u_wall[k] = uw[k]
    s.nu, s.kappa_max, s.q = p.nu, p.kappa_max, p.q
    s.margin = p.margin
    s.th_min, s.th_max = p.th_min, p.th_max
    s.nt, s.r_t, s.r_w = p.nt, p.r_t, p.r_w
    s.phi = p.phi
    s.objective = p.objective
    s.w_d, s.w_t, s.l_m = p.w_d, p.w_t, p.l_m
    s.rot = getattr(p, "rot", 0)
    for k in range(2):
        s.tilt_min[k] = p.tilt_min[k]
        s.tilt_max[k] = p.tilt_max[k]
    return s


def mw(p) -> int:
    """Motion row width: 8, or 12 with three rotation angles."""
    return 12 if getattr(p, "rot", 0) == 1 else 8


def npsi(p) -> int:
    """Rotation design variables per step: 1, or 3 with three angles."""
    return 3 if getattr(p, "rot", 0) == 1 else 1


def _psi_shape(p, a):
    return a.reshape(p.nt, 3) if npsi(p) == 3 else a


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _check(rc: int, name: str):
    if rc != 0:
        raise ValueError(f"{name}: oracle rejected the problem (code {rc})")


def motion(p, chi, psi) -> np.ndarray:
    out = np.zeros((p.nt, mw(p)))
    _check(lib().orc_motion(C.byref(to_struct(p)), _ptr(_f64(chi)), _ptr(_f64(psi)),
                            _ptr(out)), "orc_motion")
    return out


def kappa_ref(p, gamma) -> np.ndarray:
    out = np.zeros(p.Mtot)
    _check(lib().orc_kappa_ref(C.byref(to_struct(p)), _ptr(_f64(gamma)), _ptr(out)),
           "orc_kappa_ref")
    return out


def map_fields(p, kref, motion8):
    k = np.zeros(p.N)
    us = np.zeros(p.d * p.N)
    _check(lib().orc_map(C.byref(to_struct(p)), _ptr(_f64(kref)), _ptr(_f64(motion8)),
                         _ptr(k), _ptr(us)), "orc_map")
    return k, us


def map_adjoint(p, kref, motion8, kbar, usbar, kref_bar=None):
    kb = np.zeros(p.Mtot) if kref_bar is None else kref_bar
    mb = np.zeros(mw(p))
    _check(lib().orc_map_adjoint(C.byref(to_struct(p)), _ptr(_f64(kref)), _ptr(_f64(motion8)),
                                 _ptr(_f64(kbar)), _ptr(_f64(usbar)), _ptr(kb), _ptr(mb)),
           "orc_map_adjoint")
    return kb, mb


def step(p, state, kappa, us) -> np.ndarray:
    out = np.zeros((p.d + 1) * p.N)
    _check(lib().orc_step(C.byref(to_struct(p)), _ptr(_f64(state)), _ptr(_f64(kappa)),
                          _ptr(_f64(us)), _ptr(out)), "orc_step")
    return out


def step_adjoint(p, state_in, state_out, kappa, us, lam):
    lp = np.zeros((p.d + 1) * p.N)
    kb = np.zeros(p.N)
    ub = np.zeros(p.d * p.N)
    _check(lib().orc_step_adjoint(C.byref(to_struct(p)), _ptr(_f64(state_in)),
                                  _ptr(_f64(state_out)), _ptr(_f64(kappa)), _ptr(_f64(us)),
                                  _ptr(_f64(lam)), _ptr(lp), _ptr(kb), _ptr(ub)),
           "orc_step_adjoint")
    return lp, kb, ub


def forward(p, gamma, chi, psi, state0=None, want_traj=False, want_final=True):
    J = np.zeros(3)
    S = (p.d + 1) * p.N
    fin = np.zeros(S) if want_final else None
    traj = np.zeros((p.nt + 1) * S) if want_traj else None
    _check(lib().orc_forward(C.byref(to_struct(p)), _ptr(_f64(gamma)), _ptr(_f64(chi)),
                             _ptr(_f64(psi)), _ptr(_f64(state0)), _ptr(fin), _ptr(J),
                             _ptr(traj)), "orc_forward")
    out = {"J": J[0], "E": J[1], "V": J[2], "final": fin}
    if want_traj:
        out["traj"] = traj.reshape(p.nt + 1, S)
    return out


def adjoint(p, gamma, chi, psi, state0=None, dJ=1.0, adj_terminal=None):
    S = (p.d + 1) * p.N
    ai = np.zeros(S)
    dg = np.zeros(p.M)
    dc = np.zeros(p.nt * 3)
    dp = np.zeros(p.nt * npsi(p))
    kb = np.zeros(p.Mtot)
    mb = np.zeros(p.nt * mw(p))
    _check(lib().orc_adjoint(C.byref(to_struct(p)), _ptr(_f64(gamma)), _ptr(_f64(chi)),
                             _ptr(_f64(psi)), _ptr(_f64(state0)), C.c_double(dJ),
                             _ptr(_f64(adj_terminal)), _ptr(ai), _ptr(dg), _ptr(dc), _ptr(dp),
                             _ptr(kb), _ptr(mb)), "orc_adjoint")
    return {"adj_initial": ai, "dgamma": dg, "dchi": dc.reshape(p.nt, 3), "dpsi": _psi_shape(p, dp),
            "kref_bar": kb, "motion_bar": mb.reshape(p.nt, mw(p))}


def alks_state_size(p) -> int:
    """Values of the ALKS adj_initial / adj_terminal: the dJ/d(state0)
    estimate [d+1][N], then p~ [N], u~ [d][N] and the symmetric s~
    [d(d+1)/2][N]."""
    return (p.d + 1 + 1 + p.d + p.d * (p.d + 1) // 2) * p.N


def alks_adjoint(p, gamma, chi, psi, state0=None, dJ=1.0, adj_terminal=None):
    """Paper-literal ALKS backward (Sec. 2.5); outputs as adjoint(), with
    adj_initial of alks_state_size(p) values (the dJ/d(state0) estimate, then
    the ALKS state p~, u~, s~ of level 0); adj_terminal: the same layout,
    carried from an earlier run (Algorithm 1's periodic approximation)."""
    S = alks_state_size(p)
    ai = np.zeros(S)
    dg = np.zeros(p.M)
    dc = np.zeros(p.nt * 3)
    dp = np.zeros(p.nt * npsi(p))
    kb = np.zeros(p.Mtot)
    mb = np.zeros(p.nt * mw(p))
    _check(lib().orc_alks_adjoint(C.byref(to_struct(p)), _ptr(_f64(gamma)), _ptr(_f64(chi)),
                                  _ptr(_f64(psi)), _ptr(_f64(state0)), C.c_double(dJ),
                                  _ptr(_f64(adj_terminal)), _ptr(ai), _ptr(dg), _ptr(dc),
                                  _ptr(dp), _ptr(kb), _ptr(mb)),
           "orc_alks_adjoint")
    return {"adj_initial": ai, "dgamma": dg, "dchi": dc.reshape(p.nt, 3), "dpsi": _psi_shape(p, dp),
            "kref_bar": kb, "motion_bar": mb.reshape(p.nt, mw(p))}


def alks_vector(p, carry, u):
    """V of the ALKS adjoint equilibrium for carry = (p~, u~, symmetric s~)
    [(1 + d + d(d+1)/2)][N] and the level's velocity u [d][N]."""
    out = np.zeros(p.d * p.N)
    _check(lib().orc_alks_vector(C.byref(to_struct(p)), _ptr(_f64(carry)), _ptr(_f64(u)),
                                 _ptr(out)), "orc_alks_vector")
    return out


def j2_sums(p, kref, motion8, u):
    """Unnormalised J2 step sums (sum f_1, u^G_2 sum f_2, omega sum v x f) of
    the fluid velocity u [2][N] at one step's motion (Eq. objective2)."""
    out = np.zeros(3)
    _check(lib().orc_j2_sums(C.byref(to_struct(p)), _ptr(_f64(kref)), _ptr(_f64(motion8)),
                             _ptr(_f64(u)), _ptr(out)), "orc_j2_sums")
    return out


def alks_gather(p, fields_next, u_next):
    """One source-free ALKS level: (p~, u~ [d], s~ [9]) planes of level t+1 and
    u of level t+1 -> the gathered moments of level t, same [1+d+9][N] layout."""
    out = np.zeros((1 + p.d + 9) * p.N)
    _check(lib().orc_alks_gather(C.byref(to_struct(p)), _ptr(_f64(fields_next)),
                                 _ptr(_f64(u_next)), _ptr(out)), "orc_alks_gather")
    return out


def design_prelude(p, gamma, radius, beta, eta):
    """Density filter and Heaviside projection (Sec. 3.1) on the inner design grid."""
    out = np.zeros(p.M)
    _check(lib().orc_design_prelude(C.byref(to_struct(p)), _ptr(_f64(gamma)), C.c_double(radius),
                                    C.c_double(beta), C.c_double(eta), _ptr(out)),
           "orc_design_prelude")
    return out


def design_prelude_adjoint(p, gamma, radius, beta, eta, dphys):
    out = np.zeros(p.M)
    _check(lib().orc_design_prelude_adjoint(C.byref(to_struct(p)), _ptr(_f64(gamma)),
                                            C.c_double(radius), C.c_double(beta),
                                            C.c_double(eta), _ptr(_f64(dphys)), _ptr(out)),
           "orc_design_prelude_adjoint")
    return out


def constraints(p, phys, chi, psi, vmax, omega_max, p_omega):
    """(G1, G2, G3) of Sec. 2.6 with dG1, dG2 [M] and dG3/dpsi [nt]."""
    G = np.zeros(3)
    d1, d2, d3 = np.zeros(p.M), np.zeros(p.M), np.zeros(p.nt * npsi(p))
    _check(lib().orc_constraints(C.byref(to_struct(p)), _ptr(_f64(phys)), _ptr(_f64(chi)),
                                 _ptr(_f64(psi)), C.c_double(vmax), C.c_double(omega_max),
                                 C.c_double(p_omega), _ptr(G), _ptr(d1), _ptr(d2), _ptr(d3)),
           "orc_constraints")
    return G, d1, d2, d3


def sensitivities(p, gamma, kref_bar, motion_bar):
    dg = np.zeros(p.M)
    dc = np.zeros(p.nt * 3)
    dp = np.zeros(p.nt * npsi(p))
    _check(lib().orc_sensitivities(C.byref(to_struct(p)), _ptr(_f64(gamma)),
                                   _ptr(_f64(kref_bar)), _ptr(_f64(motion_bar)), None,
                                   _ptr(dg), _ptr(dc), _ptr(dp)), "orc_sensitivities")
    return dg, dc.reshape(p.nt, 3), dp


def forward_cs(p, gamma, chi, psi, dgamma=None, dchi=None, dpsi=None, state0=None,
               dstate0=None, h=1e-30):
    """Complex-step derivative: returns (J3, dJ3) with dJ3 = Im J(x + i h v) / h."""
    Jr = np.zeros(3)
    Ji = np.zeros(3)
    sc = (lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64) * h)
    _check(lib().orc_forward_cs(C.byref(to_struct(p)), _ptr(_f64(gamma)), _ptr(sc(dgamma)),
                                _ptr(_f64(chi)), _ptr(sc(dchi)), _ptr(_f64(psi)), _ptr(sc(dpsi)),
                                _ptr(_f64(state0)), _ptr(sc(dstate0)), _ptr(Jr), _ptr(Ji)),
           "orc_forward_cs")
    return Jr, Ji / h


def step_cs(p, state, kappa, us, dstate=None, dkappa=None, dus=None, h=1e-30):
    S = (p.d + 1) * p.N
    out_r = np.zeros(S)
    out_i = np.zeros(S)
    sc = (lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64) * h)
    _check(lib().orc_step_cs(C.byref(to_struct(p)), _ptr(_f64(state)), _ptr(sc(dstate)),
                             _ptr(_f64(kappa)), _ptr(sc(dkappa)), _ptr(_f64(us)), _ptr(sc(dus)),
                             _ptr(out_r), _ptr(out_i)), "orc_step_cs")
    return out_r, out_i / h


def map_cs(p, kref, motion8, dkref=None, dmotion8=None, h=1e-30):
    kr, ki = np.zeros(p.N), np.zeros(p.N)
    ur, ui = np.zeros(p.d * p.N), np.zeros(p.d * p.N)
    sc = (lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64) * h)
    _check(lib().orc_map_cs(C.byref(to_struct(p)), _ptr(_f64(kref)), _ptr(sc(dkref)),
                            _ptr(_f64(motion8)), _ptr(sc(dmotion8)), _ptr(kr), _ptr(ki),
                            _ptr(ur), _ptr(ui)), "orc_map_cs")
    return kr, ki / h, ur, ui / h
