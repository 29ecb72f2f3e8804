"""ctypes view of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product package never imports it.

Arrays cross as numpy float64 in the oracle's own layout:
state ``(nz, ny, nx, 2, 19)``, densities ``(nz, ny, nx, 2)``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of the same source (the sanitizer build of
# the sanitized test run); by default the optimised liboracle.so
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

CA_NO_REF = 1
CA_E1_FLAT = 2
CA_E2_FLAT = 4
CA_RAY_LIMIT = 8
CA_NO_APEX = 16
CA_NO_DROP = 32
CA_E2_EMPTY = 64
CA_E2_WHOLE_LAYER = 128


class OraParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("psi", ctypes.c_int32),
        ("tau", ctypes.c_double * 2),
        ("g_ab", ctypes.c_double),
        ("g_wall", ctypes.c_double * 2),
        ("rho_wall", ctypes.c_double * 2),
        ("w_axis", ctypes.c_double), ("w_diag", ctypes.c_double),
    ]


class OraCaCfg(ctypes.Structure):
    _fields_ = [
        ("ic", ctypes.c_int32), ("jc", ctypes.c_int32),
        ("z_solid_top", ctypes.c_int32), ("offset", ctypes.c_int32),
        ("eps", ctypes.c_double),
    ]


class OraCa(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "theta_e1", "h_e1", "a_e1", "R_e1", "aref_e1", "H_e1",
        "theta_e2", "h_e2", "a_e2", "R_e2", "aref_e2", "H_e2", "cx", "cy")] + [
        ("flags", ctypes.c_int32), ("pad", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_ if n != "pad"}


def build():
    """Compile liboracle.so with the oracle's own Makefile."""
    subprocess.run(["make", "-s", "-C", _HERE, "-B", "liboracle.so"], check=True)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            if "ORACLE_LIB" in os.environ:
                raise FileNotFoundError(_LIB_PATH)
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.ora_create.restype = vp
        L.ora_create.argtypes = [ctypes.POINTER(OraParams), vp]
        L.ora_destroy.argtypes = [vp]
        L.ora_set_params.argtypes = [vp, ctypes.POINTER(OraParams)]
        L.ora_init_equilibrium.argtypes = [vp, dp, dp]
        L.ora_init_equilibrium_u.argtypes = [vp, dp, dp, dp]
        L.ora_step.argtypes = [vp, ctypes.c_int64]
        L.ora_step_count.restype = ctypes.c_int64
        L.ora_step_count.argtypes = [vp]
        L.ora_get_state.argtypes = [vp, dp]
        L.ora_set_state.argtypes = [vp, dp]
        L.ora_density.argtypes = [vp, dp]
        L.ora_observables.argtypes = [vp, dp]
        L.ora_stream.argtypes = [vp, dp, dp]
        L.ora_force.argtypes = [vp, dp, dp]
        L.ora_contact_angle.argtypes = [vp, ctypes.POINTER(OraCaCfg), ctypes.POINTER(OraCa)]
        L.ora_contact_angle_phi.argtypes = [vp, ctypes.POINTER(OraCaCfg), dp, ctypes.POINTER(OraCa)]
        L.ora_ca_seed.argtypes = [vp, ctypes.POINTER(OraCaCfg), ctypes.c_double, dp]
        L.ora_adjoint_step.argtypes = [vp, dp, dp, dp]
        L.ora_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.ora_tables.argtypes = [ctypes.POINTER(ctypes.c_int32), dp, ctypes.POINTER(ctypes.c_int32)]
        L.ora_pressure_tensor.argtypes = [vp, dp]
        L.ora_radial_tension.restype = ctypes.c_double
        L.ora_radial_tension.argtypes = [vp, dp, ctypes.c_double, ctypes.c_int32, dp, dp, dp]
        L.ora_radial_tension_axes.restype = ctypes.c_double
        L.ora_radial_tension_axes.argtypes = [vp, dp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                              dp, dp, dp]
        L.ora_young_angle.restype = ctypes.c_double
        L.ora_young_angle.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.ora_huang_angle.restype = ctypes.c_double
        L.ora_huang_angle.argtypes = [ctypes.POINTER(OraParams), ctypes.c_double, ctypes.c_double]
        L.ora_surface_tension_z.restype = ctypes.c_double
        L.ora_surface_tension_z.argtypes = [vp, dp]
        L.ora_num_threads.restype = ctypes.c_int
        L.ora_num_threads.argtypes = []
        L.ora_set_threads.restype = None
        L.ora_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tables():
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    lib().ora_tables(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(w),
                     opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return c, w, opp


def equilibrium(rho, u):
    out = np.zeros(19)
    uu = np.ascontiguousarray(u, np.float64)
    lib().ora_equilibrium(float(rho), _dp(uu), _dp(out))
    return out


def make_params(p):
    """OraParams from a dict with the keys of ``workloads.params``."""
    op = OraParams()
    op.nx, op.ny, op.nz = p["nx"], p["ny"], p["nz"]
    op.psi = p.get("psi", 0)
    op.tau[0], op.tau[1] = p["tau"]
    op.g_ab = p["g_ab"]
    op.g_wall[0], op.g_wall[1] = p["g_wall"]
    op.rho_wall[0], op.rho_wall[1] = p["rho_wall"]
    op.w_axis = p.get("w_axis", 1.0)
    op.w_diag = p.get("w_diag", 1.0)
    return op


def make_ca_cfg(c):
    cfg = OraCaCfg()
    cfg.ic, cfg.jc = c["ic"], c["jc"]
    cfg.z_solid_top, cfg.offset = c["z_solid_top"], c["offset"]
    cfg.eps = c.get("eps", 0.2)
    return cfg


class Lattice:
    """One oracle lattice.  ``solid`` is a uint8 array of shape (nz, ny, nx)."""

    def __init__(self, params, solid=None):
        self.p = dict(params)
        self.shape = (params["nz"], params["ny"], params["nx"])
        self.N = int(np.prod(self.shape))
        if solid is None:
            solid = np.zeros(self.shape, np.uint8)
        self.solid = np.ascontiguousarray(solid, np.uint8).reshape(self.shape)
        self._op = make_params(params)
        self._h = lib().ora_create(ctypes.byref(self._op), self.solid.ctypes.data)
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().ora_destroy(self._h)
            self._h = None

    def set_params(self, params):
        op = make_params(params)
        if lib().ora_set_params(self._h, ctypes.byref(op)) != 0:
            raise ValueError("oracle rejected the parameters")
        self.p = dict(params)
        self._op = op

    def init_equilibrium(self, rho_a, rho_b, u=None):
        ra = np.ascontiguousarray(rho_a, np.float64).reshape(self.shape)
        rb = np.ascontiguousarray(rho_b, np.float64).reshape(self.shape)
        if u is None:
            lib().ora_init_equilibrium(self._h, _dp(ra), _dp(rb))
        else:
            uu = np.ascontiguousarray(u, np.float64).reshape(self.shape + (3,))
            lib().ora_init_equilibrium_u(self._h, _dp(ra), _dp(rb), _dp(uu))

    def step(self, n=1):
        lib().ora_step(self._h, int(n))

    @property
    def step_count(self):
        return lib().ora_step_count(self._h)

    def get_state(self):
        s = np.zeros(self.shape + (2, 19))
        lib().ora_get_state(self._h, _dp(s))
        return s

    def set_state(self, s):
        s = np.ascontiguousarray(s, np.float64).reshape(self.shape + (2, 19))
        lib().ora_set_state(self._h, _dp(s))

    def density(self):
        r = np.zeros(self.shape + (2,))
        lib().ora_density(self._h, _dp(r))
        return r

    def observables(self):
        o = np.zeros(6)
        lib().ora_observables(self._h, _dp(o))
        return {"mass": (o[0], o[1]), "momentum": (o[2], o[3], o[4]), "finite": bool(o[5])}

    def stream(self, f):
        f = np.ascontiguousarray(f, np.float64).reshape(self.shape + (2, 19))
        out = np.zeros_like(f)
        lib().ora_stream(self._h, _dp(f), _dp(out))
        return out

    def force(self, rho):
        r = np.ascontiguousarray(rho, np.float64).reshape(self.shape + (2,))
        F = np.zeros(self.shape + (2, 3))
        lib().ora_force(self._h, _dp(r), _dp(F))
        return F

    def pressure_tensor(self):
        """(nz, ny, nx, 6): xx, yy, zz, xy, xz, yz; zero at solid nodes."""
        P = np.zeros(self.shape + (6,))
        lib().ora_pressure_tensor(self._h, _dp(P))
        return P

    def surface_tension_z(self):
        """(sum over planes of <P_zz - (P_xx + P_yy)/2>, plane profile)."""
        prof = np.zeros(self.shape[0])
        g = lib().ora_surface_tension_z(self._h, _dp(prof))
        return g, prof

    def radial_tension(self, center, rmax, nbins, periodic=(True, True, True)):
        """(gamma, R_s, profile of P_N - P_T, profile of phi) about center;
        periodic: per axis, whether distances take the minimum image."""
        c = np.ascontiguousarray(center, np.float64)
        prof = np.zeros(nbins)
        pphi = np.zeros(nbins)
        rs = np.zeros(1)
        mask = sum(1 << a for a in range(3) if periodic[a])
        g = lib().ora_radial_tension_axes(self._h, _dp(c), mask, float(rmax), int(nbins), _dp(prof),
                                          _dp(pphi), _dp(rs))
        return g, rs[0], prof, pphi

    def contact_angle(self, cfg):
        out = OraCa()
        c = make_ca_cfg(cfg)
        rc = lib().ora_contact_angle(self._h, ctypes.byref(c), ctypes.byref(out))
        d = out.as_dict()
        d["status"] = rc
        return d

    def contact_angle_phi(self, cfg, phi):
        out = OraCa()
        c = make_ca_cfg(cfg)
        ph = np.ascontiguousarray(phi, np.float64).reshape(self.shape)
        rc = lib().ora_contact_angle_phi(self._h, ctypes.byref(c), _dp(ph), ctypes.byref(out))
        d = out.as_dict()
        d["status"] = rc
        return d

    def ca_seed(self, cfg, dL_dtheta=1.0):
        lam = np.zeros(self.shape + (2, 19))
        c = make_ca_cfg(cfg)
        rc = lib().ora_ca_seed(self._h, ctypes.byref(c), float(dL_dtheta), _dp(lam))
        return lam, rc

    def adjoint_step(self, state_t, lam):
        st = np.ascontiguousarray(state_t, np.float64).reshape(self.shape + (2, 19))
        lm = np.array(lam, np.float64, copy=True).reshape(self.shape + (2, 19))
        dp = np.zeros(5)
        lib().ora_adjoint_step(self._h, _dp(st), _dp(lm), _dp(dp))
        return lm, dp


def num_threads():
    """Host threads the oracle's per-node loops use."""
    return lib().ora_num_threads()


def set_threads(n):
    """Use n host threads (results are independent of the count)."""
    lib().ora_set_threads(int(n))


def young_angle(gamma_sg, gamma_sl, gamma_lg):
    return lib().ora_young_angle(float(gamma_sg), float(gamma_sl), float(gamma_lg))


def huang_angle(params, rho_in, rho_out):
    op = make_params(params)
    return lib().ora_huang_angle(ctypes.byref(op), float(rho_in), float(rho_out))


def to_gpu_layout(state):
    """(nz, ny, nx, 2, 19) oracle state -> (2, 19, nz, ny, nx) structure of arrays."""
    return np.ascontiguousarray(np.transpose(state, (3, 4, 0, 1, 2)))


def from_gpu_layout(state):
    """(2, 19, nz, ny, nx) -> (nz, ny, nx, 2, 19)."""
    return np.ascontiguousarray(np.transpose(state, (2, 3, 4, 0, 1)))


def theta_e2_gradient_run(params, solid, rho_a, rho_b, nsteps, cfg, target_deg):
    """Loss (theta_E2 - target)^2 in deg^2 after nsteps and its exact gradient
    with respect to (rho_wall_A, rho_wall_B, g_ab, g_wall_A, g_wall_B), by
    storing every state and running the adjoint steps backwards."""
    L = Lattice(params, solid)
    L.init_equilibrium(rho_a, rho_b)
    states = []
    for _ in range(nsteps):
        states.append(L.get_state())
        L.step(1)
    ca = L.contact_angle(cfg)
    theta = ca["theta_e2"]
    loss = (theta - target_deg) ** 2
    dL_dtheta = 2.0 * (theta - target_deg) * (180.0 / np.pi)
    lam, _ = L.ca_seed(cfg, dL_dtheta)
    grad = np.zeros(5)
    for t in range(nsteps - 1, -1, -1):
        lam, dp = L.adjoint_step(states[t], lam)
        grad += dp
    return loss, theta, grad
