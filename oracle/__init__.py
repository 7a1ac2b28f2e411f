"""FP64 CPU oracle of the D3Q27 cumulant LBM with actuator-line coupling.

TEST INFRASTRUCTURE ONLY: plain, slow, obviously-correct reference code
(written from Sec. 2.1-2.2 of the waLBerla-wind paper, arXiv 2402.13171).
Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package. It shares no code with the HIP library.

The C sources next to this file are compiled into ``liboracle.so`` by
:func:`build` (gcc, OpenMP); this module is a ctypes binding to them.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = ["orc_lattice.c", "orc_mlp.c", "orc_solver.c", "orc_alm.c", "orc_turbine.c"]

PERIODIC, INOUT, NOSLIP, FREESLIP = 0, 1, 2, 3
CLOSURE_NONE, CLOSURE_SMAG, CLOSURE_MLP = 0, 1, 2
MLP_NPARAM = 1313
MLP_NBLOB = MLP_NPARAM + 13


def build(verbose: bool = False) -> str:
    """Compile the oracle C sources into liboracle.so (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-Wall", "-Wno-unused-function", "-o", _SO]
    cmd += [os.path.join(_HERE, s) for s in _SRC] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = C.CDLL(_SO)
        _declare(_lib)
    return _lib


class Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("omega", C.c_double * 10), ("closure", C.c_int),
                ("cs", C.c_double), ("bc_x", C.c_int), ("bc_zlo", C.c_int),
                ("bc_zhi", C.c_int), ("u_in", C.c_double * 3),
                ("body_force", C.c_double * 3), ("mlp_emulate_bf16", C.c_int)]


class RotorDesc(C.Structure):
    _fields_ = [("hub", C.c_double * 3), ("radius", C.c_double),
                ("omega_rot", C.c_double), ("azimuth0", C.c_double),
                ("eps", C.c_double), ("pitch_deg", C.c_double),
                ("n_blades", C.c_int), ("n_points", C.c_int),
                ("r", C.POINTER(C.c_double)), ("chord", C.POINTER(C.c_double)),
                ("twist_deg", C.POINTER(C.c_double)), ("dl", C.POINTER(C.c_double)),
                ("n_polar", C.c_int), ("alpha_deg", C.POINTER(C.c_double)),
                ("cl", C.POINTER(C.c_double)), ("cd", C.POINTER(C.c_double)),
                ("kernel", C.c_int), ("tip_loss", C.c_int)]

KERNEL_GAUSS, KERNEL_ROMA3 = 0, 1


class NodeDesc(C.Structure):
    _fields_ = [("parent", C.c_int), ("kind", C.c_int), ("force", C.c_int),
                ("n_points", C.c_int), ("n_azimuth", C.c_int), ("tip_loss", C.c_int),
                ("pos", C.c_double * 3), ("rot", C.c_double * 9), ("axis", C.c_double * 3),
                ("omega", C.c_double), ("angle0", C.c_double),
                ("amp", C.c_double), ("freq", C.c_double), ("phase", C.c_double),
                ("disp", C.c_double * 3), ("dir", C.c_double * 3), ("normal", C.c_double * 3),
                ("coef", C.c_double), ("pitch_deg", C.c_double),
                ("s", C.POINTER(C.c_double)), ("width", C.POINTER(C.c_double)),
                ("chord", C.POINTER(C.c_double)), ("twist", C.POINTER(C.c_double))]


class TurbineDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int), ("nodes", C.POINTER(NodeDesc)),
                ("kernel", C.c_int), ("eps", C.c_double),
                ("n_blades", C.c_int), ("radius", C.c_double),
                ("n_polar", C.c_int), ("alpha_deg", C.POINTER(C.c_double)),
                ("cl", C.POINTER(C.c_double)), ("cd", C.POINTER(C.c_double))]


NODE_KIND = {"frame": 0, "line": 1, "disk": 2}
FORCE_KIND = {"none": 0, "blade": 1, "drag": 2}


_D = C.POINTER(C.c_double)


def _declare(L):
    v = None
    sig = {
        "orc_lattice": (v, [C.POINTER(C.c_int), _D]),
        "orc_feq": (v, [C.c_double, _D, _D]),
        "orc_central_moments_direct": (v, [_D, _D, _D]),
        "orc_central_moments": (v, [_D, _D, _D]),
        "orc_central_to_pops": (v, [_D, _D, _D]),
        "orc_cumulants": (v, [_D, _D]),
        "orc_cumulants_inverse": (v, [_D, _D]),
        "orc_relax": (v, [_D, _D, _D]),
        "orc_collide": (v, [_D, _D, _D, _D]),
        "orc_smagorinsky_omega": (C.c_double, [_D, C.c_double, C.c_double]),
        "orc_closure_features": (v, [_D, C.c_double, _D]),
        "orc_mlp_nu_t": (C.c_double, [_D, _D, C.c_int]),
        "orc_mlp_omega": (C.c_double, [_D, _D, C.c_double, C.c_int]),
        "orc_bf16_round": (C.c_double, [C.c_double]),
        "orc_create": (C.c_void_p, [C.POINTER(Params)]),
        "orc_destroy": (v, [C.c_void_p]),
        "orc_cells": (C.c_size_t, [C.c_void_p]),
        "orc_init_fields": (v, [C.c_void_p, _D, _D]),
        "orc_set_pops": (v, [C.c_void_p, _D]),
        "orc_get_pops": (v, [C.c_void_p, _D]),
        "orc_set_force_field": (v, [C.c_void_p, _D]),
        "orc_set_inlet_plane": (v, [C.c_void_p, _D]),
        "orc_set_mlp": (v, [C.c_void_p, _D]),
        "orc_step": (v, [C.c_void_p, C.c_int]),
        "orc_get_fields": (v, [C.c_void_p, _D, _D]),
        "orc_global_moments": (v, [C.c_void_p, _D, _D, _D]),
        "orc_time": (C.c_long, [C.c_void_p]),
        "orc_get_force": (v, [C.c_void_p, _D]),
        "orc_set_rotor": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(RotorDesc)]),
        "orc_rotor_loads": (v, [C.c_void_p, C.c_int, _D, _D]),
        "orc_rotor_points": (v, [C.c_void_p, C.c_int, _D]),
        "orc_trilinear": (v, [C.c_void_p, _D, C.c_int, _D, _D]),
        "orc_blade_element": (v, [C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_double, C.c_double, C.c_int,
                                  _D, _D, _D, _D, _D, _D]),
        "orc_spread_point": (v, [C.c_void_p, _D, _D, C.c_double, _D]),
        "orc_spread_point_roma": (v, [C.c_void_p, _D, _D, _D]),
        "orc_roma_phi": (C.c_double, [C.c_double]),
        "orc_tip_loss": (C.c_double, [C.c_int, C.c_double, C.c_double, C.c_double]),
        "orc_set_turbine": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(TurbineDesc)]),
        "orc_turbine_npoints": (C.c_int, [C.POINTER(TurbineDesc)]),
        "orc_turbine_kinematics": (C.c_int, [C.POINTER(TurbineDesc), C.c_double, _D, _D, _D]),
        "orc_turbine_loads": (v, [C.c_void_p, C.c_int, _D, _D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args


def _p(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- single cell
def lattice():
    c = np.zeros((27, 3), dtype=np.int32)
    w = np.zeros(27)
    lib().orc_lattice(c.ctypes.data_as(C.POINTER(C.c_int)), _p(w))
    return c, w


def feq(rho, u):
    f = np.zeros(27)
    lib().orc_feq(float(rho), _p(_f64(u)), _p(f))
    return f


def central_moments(f, u, direct=False):
    out = np.zeros(27)
    fn = lib().orc_central_moments_direct if direct else lib().orc_central_moments
    fn(_p(_f64(f)), _p(_f64(u)), _p(out))
    return out


def central_to_pops(kappa, u):
    out = np.zeros(27)
    lib().orc_central_to_pops(_p(_f64(kappa)), _p(_f64(u)), _p(out))
    return out


def cumulants(kappa):
    out = np.zeros(27)
    lib().orc_cumulants(_p(_f64(kappa)), _p(out))
    return out


def cumulants_inverse(C_):
    out = np.zeros(27)
    lib().orc_cumulants_inverse(_p(_f64(C_)), _p(out))
    return out


def relax(C_, omega):
    out = np.zeros(27)
    lib().orc_relax(_p(_f64(C_)), _p(_f64(omega)), _p(out))
    return out


def collide(f, F, omega):
    out = np.zeros(27)
    om = np.ones(10)
    om[: len(omega)] = omega
    lib().orc_collide(_p(_f64(f)), _p(_f64(F)), _p(om), _p(out))
    return out


def smagorinsky_omega(kappa, omega0, cs):
    return lib().orc_smagorinsky_omega(_p(_f64(kappa)), float(omega0), float(cs))


def closure_features(kappa, omega0):
    out = np.zeros(6)
    lib().orc_closure_features(_p(_f64(kappa)), float(omega0), _p(out))
    return out


def mlp_nu_t(blob, feat, emulate_bf16=False):
    return lib().orc_mlp_nu_t(_p(_f64(blob)), _p(_f64(feat)), int(emulate_bf16))


def bf16_round(x):
    return lib().orc_bf16_round(float(x))


def blade_element(rho, wn, wt, chord, dl, twist_deg, pitch_deg, polar):
    a, cl, cd = (_f64(polar[k]) for k in ("alpha_deg", "cl", "cd"))
    fn, ft, al = C.c_double(), C.c_double(), C.c_double()
    lib().orc_blade_element(float(rho), float(wn), float(wt), float(chord),
                            float(dl), float(twist_deg), float(pitch_deg), len(a),
                            _p(a), _p(cl), _p(cd), C.byref(fn), C.byref(ft),
                            C.byref(al))
    return fn.value, ft.value, al.value


def roma_phi(r):
    """The 1-D factor of the Roma et al. 3-point discrete delta."""
    return lib().orc_roma_phi(float(r))


def tip_loss(n_blades, radius, r, phi_rad):
    """Prandtl tip-loss factor (the oracle's reading of the paper's
    Glauert-type correction)."""
    return lib().orc_tip_loss(int(n_blades), float(radius), float(r), float(phi_rad))


def inflow_plane(mean, box, advect, t):
    """Inlet velocity at step t for the turbine-row case (reading: a frozen
    periodic turbulence box convected through the inlet, Taylor's
    hypothesis): mean[3, nz, ny] plus the box[3, lt, nz, ny] slice at
    s = advect * t (mod lt), linearly interpolated between slices."""
    mean = np.asarray(mean, dtype=np.float64)
    if box is None:
        return mean.copy()
    lt = box.shape[1]
    s = np.fmod(advect * t, lt)
    if s < 0:
        s += lt
    s0 = min(int(np.floor(s)), lt - 1)
    s1 = (s0 + 1) % lt
    f = s - s0
    return mean + (1.0 - f) * box[:, s0] + f * box[:, s1]


def _turbine_desc(turbine, keep):
    """ctypes description of a turbine dict (workloads.turbines format)."""
    nodes = turbine["nodes"]
    arr = (NodeDesc * len(nodes))()
    for k, nd in enumerate(nodes):
        d = arr[k]
        d.parent = nd.get("parent", -1)
        d.kind = NODE_KIND[nd.get("kind", "frame")]
        d.force = FORCE_KIND[nd.get("force", "none")]
        d.n_azimuth = nd.get("n_azimuth", 0)
        d.tip_loss = int(bool(nd.get("tip_loss", False)))
        rot = np.asarray(nd.get("rot", np.eye(3)), dtype=np.float64).reshape(9)
        for a in range(9):
            d.rot[a] = rot[a]
        for name in ("pos", "axis", "disp", "dir", "normal"):
            vec = nd.get(name, (0.0, 0.0, 0.0) if name != "axis" else (1.0, 0.0, 0.0))
            for a in range(3):
                getattr(d, name)[a] = vec[a]
        for name in ("omega", "angle0", "amp", "freq", "phase", "coef", "pitch_deg"):
            setattr(d, name, float(nd.get(name, 0.0)))
        n = 0
        for name in ("s", "width", "chord", "twist"):
            if nd.get(name) is not None:
                a = _f64(nd[name])
                keep.append(a)
                setattr(d, name, _p(a))
                n = len(a)
        d.n_points = n
    keep.append(arr)
    t = TurbineDesc()
    t.n_nodes = len(nodes)
    t.nodes = arr
    t.kernel = {"gauss": KERNEL_GAUSS, "roma3": KERNEL_ROMA3}[turbine.get("kernel", "gauss")]
    t.eps = float(turbine.get("eps", 2.0))
    t.n_blades = int(turbine.get("n_blades", 0))
    t.radius = float(turbine.get("radius", 0.0))
    pol = turbine.get("polar")
    if pol is not None:
        pa = {k: _f64(pol[k]) for k in ("alpha_deg", "cl", "cd")}
        keep += list(pa.values())
        t.n_polar = len(pa["alpha_deg"])
        t.alpha_deg, t.cl, t.cd = _p(pa["alpha_deg"]), _p(pa["cl"]), _p(pa["cd"])
    return t


def turbine_kinematics(turbine, t):
    """Positions x[npts][3], velocities v[npts][3] and node frames
    [n_nodes][15] (T row-major, origin, angular velocity) at time t."""
    keep = []
    d = _turbine_desc(turbine, keep)
    n = lib().orc_turbine_npoints(C.byref(d))
    x, v = np.zeros((n, 3)), np.zeros((n, 3))
    fr = np.zeros((d.n_nodes, 15))
    if lib().orc_turbine_kinematics(C.byref(d), float(t), _p(x), _p(v), _p(fr)) != 0:
        raise ValueError("oracle: bad turbine")
    return x, v, fr


# ---------------------------------------------------------------- domain solver
class Grid:
    """Two-array FP64 solver on an nx x ny x nz box (x fastest)."""

    def __init__(self, nx, ny, nz, omega=1.9, omega_hi=None, closure=CLOSURE_NONE,
                 cs=0.1, bc_x=PERIODIC, bc_zlo=PERIODIC, bc_zhi=PERIODIC,
                 u_in=(0.0, 0.0, 0.0), body_force=(0.0, 0.0, 0.0),
                 mlp_emulate_bf16=False):
        p = Params()
        p.nx, p.ny, p.nz = nx, ny, nz
        om = [omega] + list(omega_hi if omega_hi is not None else [1.0] * 9)
        for k in range(10):
            p.omega[k] = om[k]
        p.closure, p.cs = closure, cs
        p.bc_x, p.bc_zlo, p.bc_zhi = bc_x, bc_zlo, bc_zhi
        for k in range(3):
            p.u_in[k] = u_in[k]
            p.body_force[k] = body_force[k]
        p.mlp_emulate_bf16 = int(mlp_emulate_bf16)
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        self._h = lib().orc_create(C.byref(p))
        if not self._h:
            raise ValueError("oracle: invalid grid parameters")
        self._keep = []

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def init_fields(self, rho, u):
        rho = _f64(np.broadcast_to(rho, self.shape)).reshape(-1)
        u = _f64(u).reshape(3, -1)
        lib().orc_init_fields(self._h, _p(rho), _p(u))

    def set_pops(self, f):
        lib().orc_set_pops(self._h, _p(_f64(f).reshape(-1)))

    def get_pops(self):
        f = np.zeros((27,) + self.shape)
        lib().orc_get_pops(self._h, _p(f))
        return f

    def set_force_field(self, F):
        lib().orc_set_force_field(self._h, _p(_f64(F).reshape(-1)))

    def set_inlet_plane(self, u):
        lib().orc_set_inlet_plane(self._h, _p(_f64(u).reshape(-1)))

    def set_mlp(self, blob):
        b = _f64(blob)
        assert b.size == MLP_NBLOB
        lib().orc_set_mlp(self._h, _p(b))

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    @property
    def time(self):
        return lib().orc_time(self._h)

    def fields(self):
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        lib().orc_get_fields(self._h, _p(rho), _p(u))
        return rho, u

    def force(self):
        F = np.zeros((3,) + self.shape)
        lib().orc_get_force(self._h, _p(F))
        return F

    def global_moments(self):
        m, mom, e = C.c_double(), np.zeros(3), C.c_double()
        lib().orc_global_moments(self._h, C.byref(m), _p(mom), C.byref(e))
        return m.value, mom, e.value

    def set_rotor(self, rid, rotor):
        """rotor: dict as produced by workloads.rotor (hub, radius, ...)."""
        arrs = {k: _f64(rotor[k]) for k in ("r", "chord", "twist_deg", "dl")}
        pol = {k: _f64(rotor["polar"][k]) for k in ("alpha_deg", "cl", "cd")}
        self._keep += list(arrs.values()) + list(pol.values())
        d = RotorDesc()
        for k in range(3):
            d.hub[k] = rotor["hub"][k]
        d.radius = rotor["radius"]
        d.omega_rot = rotor["omega_rot"]
        d.azimuth0 = rotor.get("azimuth0", 0.0)
        d.eps = rotor["eps"]
        d.pitch_deg = rotor.get("pitch_deg", 0.0)
        d.n_blades = rotor["n_blades"]
        d.n_points = len(arrs["r"])
        d.r, d.chord = _p(arrs["r"]), _p(arrs["chord"])
        d.twist_deg, d.dl = _p(arrs["twist_deg"]), _p(arrs["dl"])
        d.n_polar = len(pol["alpha_deg"])
        d.alpha_deg, d.cl, d.cd = _p(pol["alpha_deg"]), _p(pol["cl"]), _p(pol["cd"])
        d.kernel = {"gauss": KERNEL_GAUSS, "roma3": KERNEL_ROMA3}[rotor.get("kernel", "gauss")]
        d.tip_loss = int(bool(rotor.get("tip_loss", False)))
        if lib().orc_set_rotor(self._h, rid, C.byref(d)) != 0:
            raise ValueError("oracle: bad rotor")
        self._rotor_np = getattr(self, "_rotor_np", {})
        self._rotor_np[rid] = rotor["n_blades"] * len(arrs["r"])

    def rotor_loads(self, rid, with_points=False):
        out = np.zeros(3)
        npts = self._rotor_np[rid]
        pf = np.zeros((npts, 3))
        lib().orc_rotor_loads(self._h, rid, _p(out), _p(pf))
        return (out, pf) if with_points else out

    def rotor_points(self, rid):
        pos = np.zeros((self._rotor_np[rid], 3))
        lib().orc_rotor_points(self._h, rid, _p(pos))
        return pos

    def set_turbine(self, tid, turbine):
        """turbine: dict as produced by workloads.turbines."""
        keep = []
        d = _turbine_desc(turbine, keep)
        if lib().orc_set_turbine(self._h, tid, C.byref(d)) != 0:
            raise ValueError("oracle: bad turbine")
        self._keep += keep
        self._turb = getattr(self, "_turb", {})
        self._turb[tid] = (d.n_nodes, lib().orc_turbine_npoints(C.byref(d)))

    def turbine_loads(self, tid):
        """(node_loads[n_nodes][7]: F, M about the node origin, P;
        points[npts][9]: x, v, F) of the last step."""
        nn, npts = self._turb[tid]
        nl, pts = np.zeros((nn, 7)), np.zeros((npts, 9))
        lib().orc_turbine_loads(self._h, tid, _p(nl), _p(pts))
        return nl, pts

    def trilinear(self, field, x):
        field = _f64(field)
        ncomp = field.size // self.n
        out = np.zeros(ncomp)
        lib().orc_trilinear(self._h, _p(field.reshape(-1)), ncomp, _p(_f64(x)), _p(out))
        return out

    def spread_point(self, xp, Fp, eps, kernel="gauss"):
        F = np.zeros((3,) + self.shape)
        if kernel == "roma3":
            lib().orc_spread_point_roma(self._h, _p(_f64(xp)), _p(_f64(Fp)), _p(F))
        else:
            lib().orc_spread_point(self._h, _p(_f64(xp)), _p(_f64(Fp)), float(eps), _p(F))
        return F
