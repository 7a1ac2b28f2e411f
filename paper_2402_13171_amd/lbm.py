"""ctypes binding of liblbm.so (the C ABI in include/lbm.h) and a small
wrapper that allocates the caller-owned device buffers through PyTorch.

Argument marshalling only: every step of the computation runs in the HIP
library. If the library has not been built this module raises on first use.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "liblbm.so")

OK, EINVAL, ENOMEM, EHIP, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
CLOSURE = {"none": 0, "smag": 1, "mlp": 2}
BC = {"periodic": 0, "inout": 1, "noslip": 2, "freeslip": 3}
MLP_NBLOB = 1326

EXPORTS = [
    "lbm_create", "lbm_destroy", "lbm_required_bytes", "lbm_attach", "lbm_init_tgv",
    "lbm_init_fields", "lbm_set_rotor", "lbm_set_inflow", "lbm_step", "lbm_get_fields", "lbm_rotor_loads",
    "lbm_global_moments", "lbm_get_pops", "lbm_sample_pops", "lbm_get_filtered", "lbm_time", "lbm_set_force_field",
    "lbm_set_closure_weights", "lbm_state_bytes", "lbm_get_state", "lbm_set_state",
    "lbm_strerror", "lbm_last_error", "lbm_copy_probe", "lbm_pattern_probe",
    "lbm_mlp_create", "lbm_mlp_destroy", "lbm_mlp_set_params", "lbm_mlp_get_params",
    "lbm_mlp_forward", "lbm_mlp_loss_grad", "lbm_mlp_loss_grad_noalloc", "lbm_mlp_adam_step", "lbm_mlp_take_loss",
    "lbm_mlp_last_error", "lbm_set_turbine", "lbm_turbine_loads", "lbm_turbine_points", "lbm_turbine_box",
]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("omega", C.c_double), ("omega_hi", C.c_double * 9),
                ("storage", C.c_int), ("closure", C.c_int), ("cs_smag", C.c_double),
                ("bc_x", C.c_int), ("bc_z_lo", C.c_int), ("bc_z_hi", C.c_int),
                ("u_in", C.c_double * 3), ("body_force", C.c_double * 3),
                ("check_every", C.c_int), ("stream", C.c_void_p), ("general_path", C.c_int),
                ("rounding", C.c_int)]


_D = C.POINTER(C.c_double)


class Rotor(C.Structure):
    _fields_ = [("hub", C.c_double * 3), ("axis", C.c_double * 3),
                ("radius", C.c_double), ("omega_rot", C.c_double), ("azimuth0", C.c_double),
                ("eps", C.c_double), ("pitch_deg", C.c_double),
                ("n_blades", C.c_int), ("n_points", C.c_int),
                ("r", _D), ("chord", _D), ("twist_deg", _D), ("dl", _D),
                ("n_polar", C.c_int), ("alpha_deg", _D), ("cl", _D), ("cd", _D),
                ("kernel", C.c_int), ("tip_loss", C.c_int)]


KERNELS = {"gauss": 0, "roma3": 1}
ROUNDING = {"stochastic": 0, "nearest": 1}


class Node(C.Structure):
    _fields_ = [("parent", C.c_int), ("kind", C.c_int), ("force", C.c_int),
                ("n_points", C.c_int), ("n_azimuth", C.c_int), ("tip_loss", C.c_int),
                ("pos", C.c_double * 3), ("rot", C.c_double * 9), ("axis", C.c_double * 3),
                ("omega", C.c_double), ("angle0", C.c_double),
                ("amp", C.c_double), ("freq", C.c_double), ("phase", C.c_double),
                ("disp", C.c_double * 3), ("dir", C.c_double * 3), ("normal", C.c_double * 3),
                ("coef", C.c_double), ("pitch_deg", C.c_double),
                ("s", _D), ("width", _D), ("chord", _D), ("twist", _D)]


class Turbine(C.Structure):
    _fields_ = [("n_nodes", C.c_int), ("nodes", C.POINTER(Node)),
                ("kernel", C.c_int), ("eps", C.c_double),
                ("n_blades", C.c_int), ("radius", C.c_double),
                ("n_polar", C.c_int), ("alpha_deg", _D), ("cl", _D), ("cd", _D)]


NODE_KINDS = {"frame": 0, "line": 1, "disk": 2}
FORCE_MODELS = {"none": 0, "blade": 1, "drag": 2}


_lib = None


def lib():
    """Load liblbm.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        raise RuntimeError(f"{SO_PATH} is not built; run __graft_entry__.build() "
                           "or python paper_2402_13171_amd/build.py")
    L = C.CDLL(SO_PATH)
    vp, i, sz = C.c_void_p, C.c_int, C.c_size_t
    sig = {
        "lbm_create": [C.POINTER(Config), C.POINTER(vp)],
        "lbm_destroy": [vp],
        "lbm_required_bytes": [vp, C.POINTER(sz), C.POINTER(sz)],
        "lbm_attach": [vp, vp, vp],
        "lbm_init_tgv": [vp, C.c_double, C.c_double, C.c_double],
        "lbm_init_fields": [vp, _D, _D],
        "lbm_set_rotor": [vp, i, C.POINTER(Rotor)],
        "lbm_set_turbine": [vp, i, C.POINTER(Turbine)],
        "lbm_turbine_loads": [vp, i, _D, _D],
        "lbm_turbine_points": [vp, i, C.POINTER(i)],
        "lbm_turbine_box": [C.POINTER(Turbine), C.POINTER(i), C.POINTER(i)],
        "lbm_step": [vp, i],
        "lbm_set_inflow": [vp, _D, _D, i, C.c_double],
        "lbm_get_fields": [vp, _D, _D],
        "lbm_rotor_loads": [vp, i, _D, _D],
        "lbm_global_moments": [vp, _D, _D, _D],
        "lbm_get_pops": [vp, _D],
        "lbm_sample_pops": [vp, C.POINTER(C.c_size_t), sz, _D],
        "lbm_get_filtered": [vp, i, _D],
        "lbm_time": [vp, C.POINTER(C.c_long)],
        "lbm_set_force_field": [vp, _D],
        "lbm_set_closure_weights": [vp, C.POINTER(C.c_float), sz],
        "lbm_state_bytes": [vp, C.POINTER(sz)],
        "lbm_get_state": [vp, vp, sz],
        "lbm_set_state": [vp, vp, sz],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    fp = C.POINTER(C.c_float)
    msig = {
        "lbm_mlp_create": [vp, C.POINTER(vp)],
        "lbm_mlp_destroy": [vp],
        "lbm_mlp_set_params": [vp, fp, sz],
        "lbm_mlp_get_params": [vp, fp, sz],
        "lbm_mlp_forward": [vp, vp, sz, vp],
        "lbm_mlp_loss_grad": [vp, vp, vp, sz, fp],
        "lbm_mlp_loss_grad_noalloc": [vp, vp, vp, sz, fp],
        "lbm_mlp_adam_step": [vp, C.c_float, C.c_float, C.c_float, C.c_float],
        "lbm_mlp_take_loss": [vp, _D],
    }
    for name, args in msig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.lbm_mlp_last_error.argtypes = [vp]
    L.lbm_mlp_last_error.restype = C.c_char_p
    L.lbm_copy_probe.argtypes = [vp, vp, sz, vp]
    L.lbm_copy_probe.restype = C.c_int
    L.lbm_pattern_probe.argtypes = [vp, C.c_int]
    L.lbm_pattern_probe.restype = C.c_int
    L.lbm_strerror.argtypes = [i]
    L.lbm_strerror.restype = C.c_char_p
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = C.c_char_p
    _lib = L
    return L


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_D)


def _turbine_struct(turbine):
    """ctypes lbm_turbine of a workloads.turbines dict, and the arrays it
    points into (keep them alive while the struct is used)."""
    nodes = turbine["nodes"]
    arr = (Node * len(nodes))()
    keep = [arr]
    for k, nd in enumerate(nodes):
        d = arr[k]
        d.parent = nd.get("parent", -1)
        d.kind = NODE_KINDS[nd.get("kind", "frame")]
        d.force = FORCE_MODELS[nd.get("force", "none")]
        d.n_azimuth = nd.get("n_azimuth", 0)
        d.tip_loss = int(bool(nd.get("tip_loss", False)))
        rot = np.asarray(nd.get("rot", np.eye(3)), dtype=np.float64).reshape(9)
        for a in range(9):
            d.rot[a] = rot[a]
        for name in ("pos", "axis", "disp", "dir", "normal"):
            vec = nd.get(name, (1.0, 0.0, 0.0) if name == "axis" else (0.0, 0.0, 0.0))
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
    t = Turbine()
    t.n_nodes, t.nodes = len(nodes), arr
    t.kernel = KERNELS[turbine.get("kernel", "gauss")]
    t.eps = float(turbine.get("eps", 2.0))
    t.n_blades = int(turbine.get("n_blades", 0))
    t.radius = float(turbine.get("radius", 0.0))
    pol = turbine.get("polar")
    if pol is not None:
        pa = {k: _f64(pol[k]) for k in ("alpha_deg", "cl", "cd")}
        keep += list(pa.values())
        t.n_polar = len(pa["alpha_deg"])
        t.alpha_deg, t.cl, t.cd = _p(pa["alpha_deg"]), _p(pa["cl"]), _p(pa["cd"])
    return t, keep


def turbine_box(turbine):
    """Inclusive lattice-node ranges (lo[3], hi[3]) of the turbine's spreading
    box (lbm_turbine_box; no device needed)."""
    t, keep = _turbine_struct(turbine)
    lo, hi = (C.c_int * 3)(), (C.c_int * 3)()
    rc = lib().lbm_turbine_box(C.byref(t), lo, hi)
    if rc != OK:
        raise LbmError(rc, lib().lbm_strerror(rc).decode())
    return list(lo), list(hi)


class Lbm:
    """One lattice on one GPU. Device memory comes from PyTorch; the library
    enqueues its kernels on a torch stream owned by this object (``stream``),
    so torch events recorded on it time the library's work."""

    def __init__(self, nx, ny, nz, omega=1.9, omega_hi=None, storage="f32", closure="none",
                 cs_smag=0.1, bc_x="periodic", bc_z=("periodic", "periodic"), u_in=(0, 0, 0),
                 body_force=(0, 0, 0), check_every=0, general_path=False, rounding="stochastic",
                 device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        cfg = Config()
        cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
        cfg.omega = omega
        for k, v in enumerate(omega_hi or []):
            cfg.omega_hi[k] = v
        cfg.storage = STORAGE[storage]
        cfg.closure = CLOSURE[closure]
        cfg.cs_smag = cs_smag
        cfg.bc_x = BC[bc_x]
        cfg.bc_z_lo, cfg.bc_z_hi = BC[bc_z[0]], BC[bc_z[1]]
        for k in range(3):
            cfg.u_in[k] = u_in[k]
            cfg.body_force[k] = body_force[k]
        cfg.check_every = check_every
        cfg.stream = self.stream.cuda_stream
        cfg.general_path = int(bool(general_path))
        cfg.rounding = ROUNDING[rounding]
        self.cfg = cfg
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        self._ctx = C.c_void_p()
        self._check(lib().lbm_create(C.byref(cfg), C.byref(self._ctx)), ctx=False)
        pb, ab = C.c_size_t(), C.c_size_t()
        self._check(lib().lbm_required_bytes(self._ctx, C.byref(pb), C.byref(ab)))
        self.pop_bytes, self.aux_bytes = pb.value, ab.value
        with torch.cuda.device(self.device):
            self.d_pops = torch.empty(self.pop_bytes, dtype=torch.uint8, device=self.device)
            self.d_aux = torch.empty(self.aux_bytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self._check(lib().lbm_attach(self._ctx, C.c_void_p(self.d_pops.data_ptr()),
                                     C.c_void_p(self.d_aux.data_ptr())))
        self._npts = {}

    # -------------------------------------------------------------- helpers
    def _check(self, rc, ctx=True):
        if rc != OK:
            msg = lib().lbm_strerror(rc).decode()
            if ctx and self._ctx:
                detail = lib().lbm_last_error(self._ctx).decode()
                if detail:
                    msg += f" ({detail})"
            raise LbmError(rc, msg)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib().lbm_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- API
    def init_tgv(self, u0=0.05, k=None, rho0=1.0):
        k = 2 * np.pi / self.cfg.nx if k is None else k
        self._check(lib().lbm_init_tgv(self._ctx, u0, k, rho0))

    def init_fields(self, rho, u):
        rho = _f64(np.broadcast_to(rho, self.shape)).reshape(-1)
        u = _f64(u).reshape(3, -1)
        self._check(lib().lbm_init_fields(self._ctx, _p(rho), _p(u)))

    def set_rotor(self, rid, rot):
        arrs = {k: _f64(rot[k]) for k in ("r", "chord", "twist_deg", "dl")}
        pol = {k: _f64(rot["polar"][k]) for k in ("alpha_deg", "cl", "cd")}
        d = Rotor()
        for k in range(3):
            d.hub[k] = rot["hub"][k]
        d.axis[0], d.axis[1], d.axis[2] = 1.0, 0.0, 0.0
        d.radius, d.omega_rot = rot["radius"], rot["omega_rot"]
        d.azimuth0, d.eps = rot.get("azimuth0", 0.0), rot["eps"]
        d.pitch_deg = rot.get("pitch_deg", 0.0)
        d.n_blades, d.n_points = rot["n_blades"], len(arrs["r"])
        d.r, d.chord = _p(arrs["r"]), _p(arrs["chord"])
        d.twist_deg, d.dl = _p(arrs["twist_deg"]), _p(arrs["dl"])
        d.n_polar = len(pol["alpha_deg"])
        d.alpha_deg, d.cl, d.cd = _p(pol["alpha_deg"]), _p(pol["cl"]), _p(pol["cd"])
        d.kernel = KERNELS[rot.get("kernel", "gauss")]
        d.tip_loss = int(bool(rot.get("tip_loss", False)))
        self._check(lib().lbm_set_rotor(self._ctx, rid, C.byref(d)))
        self._npts[rid] = d.n_blades * d.n_points

    def set_inflow(self, mean, box=None, advect=0.0):
        """mean: [3, nz, ny] inlet velocity; box: [3, lt, nz, ny] frozen
        turbulence convected at `advect` cells per step (or None)."""
        mean = _f64(mean).reshape(-1)
        if box is None:
            self._check(lib().lbm_set_inflow(self._ctx, _p(mean), None, 0, float(advect)))
        else:
            box = _f64(box)
            lt = box.shape[1]
            self._check(lib().lbm_set_inflow(self._ctx, _p(mean), _p(box.reshape(-1)), lt, float(advect)))

    def pattern_probe(self, parity):
        """One pass of the stream-collide memory traffic without the
        collision (leaves the populations permuted: initialise afterwards)."""
        self._check(lib().lbm_pattern_probe(self._ctx, int(parity)))

    def step(self, n=1):
        self._check(lib().lbm_step(self._ctx, int(n)))

    def fields(self):
        rho = np.empty(self.shape)
        u = np.empty((3,) + self.shape)
        self._check(lib().lbm_get_fields(self._ctx, _p(rho), _p(u)))
        return rho, u

    def pops(self):
        f = np.empty((27,) + self.shape)
        self._check(lib().lbm_get_pops(self._ctx, _p(f)))
        return f

    def filtered(self, w):
        """block means over w^3 cells: array [10, nz/w, ny/w, nx/w] with rho,
        ux, uy, uz, uxux, uyuy, uzuz, uxuy, uxuz, uyuz"""
        nz, ny, nx = self.shape
        out = np.empty((10, nz // w, ny // w, nx // w))
        self._check(lib().lbm_get_filtered(self._ctx, int(w), _p(out)))
        return out

    def sample_pops(self, cells):
        """populations f[m][27] of the given linear cell indices"""
        cells = np.ascontiguousarray(cells, dtype=np.uint64)
        f = np.empty((cells.size, 27))
        self._check(lib().lbm_sample_pops(self._ctx, cells.ctypes.data_as(C.POINTER(C.c_size_t)),
                                          cells.size, _p(f)))
        return f

    def set_turbine(self, tid, turbine):
        """turbine: dict of workloads.turbines (nodes with parent, kind,
        force, pose, motion and per-point arrays; kernel, eps, polars)."""
        t, keep = _turbine_struct(turbine)
        nodes = turbine["nodes"]
        self._check(lib().lbm_set_turbine(self._ctx, tid, C.byref(t)))
        npt = C.c_int()
        self._check(lib().lbm_turbine_points(self._ctx, tid, C.byref(npt)))
        self._npts[tid] = ("tree", len(nodes), npt.value)

    def turbine_loads(self, tid):
        """(node_loads[n_nodes][7]: force, moment about the node origin,
        power; points[npts][9]: x, v, F) of the last step."""
        if not isinstance(self._npts.get(tid), tuple):
            raise LbmError(EINVAL, f"slot {tid} holds no turbine tree")
        _, nn, npts = self._npts[tid]
        nl, pts = np.zeros((nn, 7)), np.zeros((npts, 9))
        self._check(lib().lbm_turbine_loads(self._ctx, tid, _p(nl), _p(pts)))
        return nl, pts

    def rotor_loads(self, rid, with_points=False):
        if isinstance(self._npts.get(rid), tuple):
            raise LbmError(EINVAL, f"slot {rid} holds a turbine tree: use turbine_loads")
        out = np.zeros(3)
        pf = np.zeros((self._npts.get(rid, 0), 3))
        self._check(lib().lbm_rotor_loads(self._ctx, rid, _p(out), _p(pf)))
        return (out, pf) if with_points else out

    def global_moments(self):
        m, e = C.c_double(), C.c_double()
        mom = np.zeros(3)
        self._check(lib().lbm_global_moments(self._ctx, C.byref(m), _p(mom), C.byref(e)))
        return m.value, mom, e.value

    @property
    def time(self):
        t = C.c_long()
        self._check(lib().lbm_time(self._ctx, C.byref(t)))
        return t.value

    def set_force_field(self, F):
        if F is None:
            self._check(lib().lbm_set_force_field(self._ctx, None))
        else:
            F = _f64(F).reshape(-1)
            self._check(lib().lbm_set_force_field(self._ctx, _p(F)))

    def set_closure_weights(self, blob):
        w = np.ascontiguousarray(blob, dtype=np.float32)
        self._check(lib().lbm_set_closure_weights(
            self._ctx, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))

    def get_state(self):
        nb = C.c_size_t()
        self._check(lib().lbm_state_bytes(self._ctx, C.byref(nb)))
        buf = np.empty(nb.value, dtype=np.uint8)
        self._check(lib().lbm_get_state(self._ctx, C.c_void_p(buf.ctypes.data), nb.value))
        return buf

    def set_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(lib().lbm_set_state(self._ctx, C.c_void_p(buf.ctypes.data), buf.size))


def copy_probe(src, dst, stream=None):
    """Device copy src -> dst (torch CUDA tensors of equal byte size) with the
    library's streaming copy kernel on `stream` (a torch stream)."""
    # the kernel reads and writes numel * element_size bytes from the base
    # pointers: both must be whole device buffers on one device
    for name, t in (("src", src), ("dst", dst)):
        if not t.is_cuda:
            raise ValueError(f"copy_probe: {name} is not a device tensor")
        if not t.is_contiguous():
            raise ValueError(f"copy_probe: {name} is not contiguous")
    if src.device != dst.device:
        raise ValueError("copy_probe: src and dst are on different devices")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("copy_probe: src and dst differ in size")
    h = stream.cuda_stream if stream is not None else None
    rc = lib().lbm_copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                              C.c_void_p(h) if h else None)
    if rc != OK:
        raise LbmError(rc, "copy probe failed")


class MlpTrainer:
    """Device-resident trainer of the closure network (lbm_mlp_* entry
    points). Batches are torch float32 CUDA tensors: features [m, 6] and
    scaled targets [m]."""

    def __init__(self, blob, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        self._h = C.c_void_p()
        rc = lib().lbm_mlp_create(C.c_void_p(self.stream.cuda_stream), C.byref(self._h))
        if rc != OK:
            raise LbmError(rc, lib().lbm_strerror(rc).decode())
        self.set_params(blob)

    def _check(self, rc):
        if rc != OK:
            raise LbmError(rc, lib().lbm_strerror(rc).decode() + " (" +
                           lib().lbm_mlp_last_error(self._h).decode() + ")")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().lbm_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, blob):
        w = np.ascontiguousarray(blob, dtype=np.float32)
        self._check(lib().lbm_mlp_set_params(self._h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))

    def get_params(self):
        w = np.empty(MLP_NBLOB, dtype=np.float32)
        self._check(lib().lbm_mlp_get_params(self._h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))
        return w

    def _sync_inputs(self, *tensors):
        # the inputs were produced on torch's current stream
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        for t in tensors:
            assert t.is_cuda and t.dtype == self.torch.float32 and t.is_contiguous()

    def forward(self, feat):
        self._sync_inputs(feat)
        out = self.torch.empty(feat.shape[0], dtype=self.torch.float32, device=self.device)
        self._check(lib().lbm_mlp_forward(self._h, C.c_void_p(feat.data_ptr()), feat.shape[0],
                                          C.c_void_p(out.data_ptr())))
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def loss_grad(self, feat, target, want_grad=False):
        self._sync_inputs(feat, target)
        g = np.empty(1313, dtype=np.float32) if want_grad else None
        gp = g.ctypes.data_as(C.POINTER(C.c_float)) if want_grad else None
        self._check(lib().lbm_mlp_loss_grad(self._h, C.c_void_p(feat.data_ptr()),
                                            C.c_void_p(target.data_ptr()), feat.shape[0], gp))
        return g

    def loss_grad_noalloc(self, feat, target, want_grad=False):
        """lbm_mlp_loss_grad_noalloc: the same result through the library's
        static scratch (no device allocation; at most 65536 samples)."""
        self._sync_inputs(feat, target)
        g = np.empty(1313, dtype=np.float32) if want_grad else None
        gp = g.ctypes.data_as(C.POINTER(C.c_float)) if want_grad else None
        self._check(lib().lbm_mlp_loss_grad_noalloc(self._h, C.c_void_p(feat.data_ptr()),
                                                    C.c_void_p(target.data_ptr()), feat.shape[0], gp))
        return g

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(lib().lbm_mlp_adam_step(self._h, lr, beta1, beta2, eps))

    def take_loss(self):
        v = C.c_double()
        self._check(lib().lbm_mlp_take_loss(self._h, C.byref(v)))
        return v.value
