"""ctypes binding of libscdrop (include/scdrop.h).

Argument marshalling only: every computation runs in the HIP library.
PyTorch provides device memory (tensors) and streams.  The library must be
built (``__graft_entry__.build()`` or ``python -m paper_0910_3915_amd.build``);
nothing here falls back to another implementation.
"""
import ctypes
import os
import re

import torch  # loaded first: libscdrop binds to the HIP runtime torch loaded

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscdrop.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "scdrop.h")

SCD_OK, SCD_EINVAL, SCD_EDEVICE, SCD_ENONFINITE, SCD_ENOINTERFACE, SCD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SCD_EDRIFT = -6
SCD_F64, SCD_F32 = 0, 1
SCD_WITH_ADJOINT = 1
CA_FLAGS = {"NO_REF": 1, "E1_FLAT": 2, "E2_FLAT": 4, "RAY_LIMIT": 8, "NO_APEX": 16,
            "NO_DROP": 32, "E2_EMPTY": 64, "E2_WHOLE_LAYER": 128}


class ScdParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("psi", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("tau", ctypes.c_double * 2), ("g_ab", ctypes.c_double),
                ("g_wall", ctypes.c_double * 2), ("rho_wall", ctypes.c_double * 2),
                ("w_axis", ctypes.c_double), ("w_diag", ctypes.c_double)]


class ScdObs(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double * 2), ("momentum", ctypes.c_double * 3),
                ("finite", ctypes.c_int32), ("pad", ctypes.c_int32), ("step", ctypes.c_int64)]


class ScdCaCfg(ctypes.Structure):
    _fields_ = [("ic", ctypes.c_int32), ("jc", ctypes.c_int32),
                ("z_solid_top", ctypes.c_int32), ("offset", ctypes.c_int32),
                ("eps", ctypes.c_double)]


class ScdCa(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "theta_e1", "h_e1", "a_e1", "R_e1", "aref_e1", "H_e1",
        "theta_e2", "h_e2", "a_e2", "R_e2", "aref_e2", "H_e2", "cx", "cy")] + [
        ("flags", ctypes.c_int32), ("pad", ctypes.c_int32)]


class ScdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"scdrop status {status}: {msg}")
        self.status = status


_lib = None

_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double
_PROTOS = {
    "scd_sizes": [ctypes.POINTER(ScdParams), ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
    "scd_create": [ctypes.POINTER(ScdParams), _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(_VP)],
    "scd_destroy": [_VP],
    "scd_set_params": [_VP, ctypes.POINTER(ScdParams)],
    "scd_set_stream": [_VP, _VP],
    "scd_init_equilibrium": [_VP, _VP, _VP],
    "scd_step": [_VP, _I64],
    "scd_get_state": [_VP, _VP],
    "scd_pop_pack": [_VP, _VP, _VP],
    "scd_pop_unpack": [_VP, _VP, _VP],
    "scd_set_state": [_VP, _VP, _I64],
    "scd_fill_state": [_VP, _D],
    "scd_density": [_VP, _VP],
    "scd_pressure_tensor": [_VP, _VP],
    "scd_radial_tension": [_VP, _VP, ctypes.POINTER(_D), _D, _I32, ctypes.POINTER(_D),
                           ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D)],
    "scd_radial_tension_axes": [_VP, _VP, ctypes.POINTER(_D), _I32, _D, _I32, ctypes.POINTER(_D),
                                ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D)],
    "scd_young_angle": [_D, _D, _D],
    "scd_huang_angle": [ctypes.POINTER(ScdParams), _D, _D],
    "scd_surface_tension_z": [_VP, _VP, ctypes.POINTER(_D), ctypes.POINTER(_D)],
    "scd_observables": [_VP, ctypes.POINTER(ScdObs)],
    "scd_set_mass_watchdog": [_VP, ctypes.c_double],
    "scd_mass_drift": [_VP, ctypes.POINTER(ctypes.c_double)],
    "scd_contact_angle": [_VP, ctypes.POINTER(ScdCaCfg), ctypes.POINTER(ScdCa)],
    "scd_contact_angle_static": [_VP, ctypes.POINTER(ScdCaCfg), ctypes.POINTER(ScdCa)],
    "scd_ca_seed": [_VP, ctypes.POINTER(ScdCaCfg), _D, _VP],
    "scd_adjoint_step": [_VP, _VP, _VP, _VP, ctypes.POINTER(_D)],
    "scd_adjoint_reset": [_VP],
    "scd_adjoint_read": [_VP, ctypes.POINTER(_D)],
    "scd_ckpt_forward": [_VP, _VP, _VP, _I64, _I64, _VP, ctypes.POINTER(ScdCaCfg), _D, ctypes.POINTER(_D)],
    "scd_ckpt_moment_cache": [_VP, _VP, _I64],
    "scd_ckpt_seg_states": [_VP, _I64, ctypes.POINTER(_I64)],
    "scd_ckpt_backward": [_VP, _I64, _I64, _VP, _VP, _VP, ctypes.POINTER(ScdCaCfg), _D, ctypes.POINTER(_D)],
    "scd_ckpt_backward2": [_VP, _I64, _I64, _I64, _VP, _VP, _VP, _VP, ctypes.POINTER(ScdCaCfg), _D,
                           ctypes.POINTER(_D)],
    "scd_tile_set": [_VP, _I32, _I32],
    "scd_tile_get": [_VP, ctypes.POINTER(_I32), ctypes.POINTER(_I32)],
    "scd_tile_list": [ctypes.POINTER(_I32), _I32, ctypes.POINTER(_I32)],
    "scd_autotune": [_VP, _I32, ctypes.c_char_p, ctypes.POINTER(_I32), ctypes.POINTER(_D)],
    "scd_graph_capture": [_VP, _I64],
    "scd_graph_replay": [_VP, _I64],
    "scd_batch_sizes": [_I32, ctypes.POINTER(ScdParams), ctypes.POINTER(ctypes.c_size_t)],
    "scd_batch_create": [_I32, ctypes.POINTER(ScdParams), ctypes.POINTER(_VP), _VP, _VP, ctypes.POINTER(_VP)],
    "scd_batch_destroy": [_VP],
    "scd_batch_lattice": [_VP, _I32, ctypes.POINTER(_VP)],
    "scd_batch_init_equilibrium": [_VP, _I32, _VP, _VP],
    "scd_batch_set_tile": [_VP, _I32, _I32, _I32],
    "scd_batch_set_member_tile": [_VP, _I32, _I32, _I32],
    "scd_batch_member_tile": [_VP, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32)],
    "scd_batch_set_blocking": [_VP, ctypes.c_int64],
    "scd_batch_blocking": [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_I32)],
    "scd_batch_step": [_VP, _I64],
    "scd_batch_graph_capture": [_VP, _I64],
    "scd_batch_graph_replay": [_VP, _I64],
    "scd_batch_autotune": [_VP, _I32, ctypes.c_char_p, ctypes.POINTER(_I32), ctypes.POINTER(_D)],
    "scd_stream_copy": [_VP, _VP, ctypes.c_size_t, _VP],
    "scd_pull_copy": [_VP],
}


def header_symbols():
    """Names of the functions that include/scdrop.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:scd_status|int64_t|double|const char\*)\s+(scd_\w+)\(", text, re.M)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _PROTOS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _I32
        L.scd_step_count.argtypes = [_VP]
        L.scd_step_count.restype = _I64
        L.scd_last_error.restype = ctypes.c_char_p
        L.scd_version.restype = ctypes.c_char_p
        L.scd_young_angle.restype = _D
        L.scd_huang_angle.restype = _D
        _lib = L
    return _lib


def check(status):
    if status != SCD_OK:
        raise ScdError(status, lib().scd_last_error().decode())
    return status


def make_params(p, adjoint=False):
    sp = ScdParams()
    sp.nx, sp.ny, sp.nz = p["nx"], p["ny"], p["nz"]
    sp.dtype = SCD_F64 if p.get("dtype", "f64") == "f64" else SCD_F32
    sp.psi = p.get("psi", 0)
    sp.flags = SCD_WITH_ADJOINT if adjoint else 0
    sp.tau[0], sp.tau[1] = p["tau"]
    sp.g_ab = p["g_ab"]
    sp.g_wall[0], sp.g_wall[1] = p["g_wall"]
    sp.rho_wall[0], sp.rho_wall[1] = p["rho_wall"]
    sp.w_axis = p.get("w_axis", 1.0)
    sp.w_diag = p.get("w_diag", 1.0)
    return sp


def make_ca_cfg(c):
    cfg = ScdCaCfg()
    cfg.ic, cfg.jc = c["ic"], c["jc"]
    cfg.z_solid_top, cfg.offset = c["z_solid_top"], c["offset"]
    cfg.eps = c.get("eps", 0.2)
    return cfg


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        return ctypes.c_void_p(None)
    return ctypes.c_void_p(stream.cuda_stream)


def _torch_dtype(sp):
    return torch.float64 if sp.dtype == SCD_F64 else torch.float32


def _alloc_bytes(nbytes, device):
    # 256-byte aligned device memory (the caching allocator aligns to 512)
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _device_f64(a, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    import numpy as np
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)


class Lattice:
    """One lattice: owns its device buffers (torch) and an scd_lattice handle."""

    def __init__(self, params, solid, device="cuda", adjoint=False, stream=None):
        self.params = dict(params)
        self.device = torch.device(device)
        self.sp = make_params(params, adjoint)
        self.shape = (params["nz"], params["ny"], params["nx"])
        self.N = params["nx"] * params["ny"] * params["nz"]
        pop_b, work_b = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib().scd_sizes(ctypes.byref(self.sp), ctypes.byref(pop_b), ctypes.byref(work_b)))
        self.pop_bytes = pop_b.value
        self.dtype = _torch_dtype(self.sp)
        self.solid = torch.as_tensor(solid, dtype=torch.uint8).reshape(self.shape).to(self.device).contiguous()
        # population buffers in the library's blocked layout (flat); zeroed so
        # that the padding slots, which nothing writes, hold zeros
        self.pop_numel = self.pop_bytes // torch.empty((), dtype=self.dtype).element_size()
        self.pop = [torch.zeros(self.pop_numel, dtype=self.dtype, device=self.device) for _ in range(2)]
        self.work = _alloc_bytes(work_b.value, self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        check(lib().scd_create(ctypes.byref(self.sp), _ptr(self.solid), _ptr(self.pop[0]), _ptr(self.pop[1]),
                               _ptr(self.work), _stream_handle(stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().scd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # Stream order: inputs made on torch's current stream are read on the
    # lattice's stream, outputs written there are read on torch's stream.
    def _after_torch(self):
        if self.stream is not None:
            self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _before_torch(self):
        if self.stream is not None:
            torch.cuda.current_stream(self.device).wait_stream(self.stream)

    # -- method calls map one to one onto the C ABI
    def set_params(self, params):
        sp = make_params(params, bool(self.sp.flags & SCD_WITH_ADJOINT))
        check(lib().scd_set_params(self.h, ctypes.byref(sp)))
        self.sp = sp
        self.params = dict(params)

    def init_equilibrium(self, rho_a, rho_b):
        ra = _device_f64(rho_a, self.device).reshape(-1)
        rb = _device_f64(rho_b, self.device).reshape(-1)
        self._after_torch()
        check(lib().scd_init_equilibrium(self.h, _ptr(ra), _ptr(rb)))
        self._keep = (ra, rb)  # alive until the kernel has read them

    def step(self, n=1):
        check(lib().scd_step(self.h, int(n)))

    @property
    def step_count(self):
        return lib().scd_step_count(self.h)

    # Population tensors: "plain" is (2, 19, nz, ny, nx), the order of the
    # Python API; "blocked" is the library's flat layout (pop_numel
    # elements), which the C calls read and write.  pack/unpack convert on
    # the lattice's stream.
    def empty_blocked(self):
        """A blocked population tensor, zeroed: the library writes only the
        node slots, so its padding slots stay zero and whole buffers compare
        and copy deterministically."""
        return torch.zeros(self.pop_numel, dtype=self.dtype, device=self.device)

    def pack(self, plain, out=None):
        plain = plain.to(device=self.device, dtype=self.dtype).contiguous()
        if plain.numel() != 2 * 19 * self.N:
            raise ValueError("plain population tensor must have 2 * 19 * N elements")
        out = self.empty_blocked() if out is None else out
        self._after_torch()
        check(lib().scd_pop_pack(self.h, _ptr(plain), _ptr(out)))
        self._before_torch()
        return out

    def unpack(self, blocked, out=None):
        if blocked.numel() != self.pop_numel:
            raise ValueError("blocked population tensor must have pop_numel elements")
        if out is None:
            out = torch.empty((2, 19) + self.shape, dtype=self.dtype, device=self.device)
        self._after_torch()
        check(lib().scd_pop_unpack(self.h, _ptr(blocked), _ptr(out)))
        self._before_torch()
        return out

    def get_state(self, out=None, blocked=False):
        b = self.empty_blocked() if (out is None or not blocked) else out
        self._after_torch()
        check(lib().scd_get_state(self.h, _ptr(b)))
        self._before_torch()
        return b if blocked else self.unpack(b, out)

    def set_state(self, src, step=0, blocked=False):
        src = src.to(device=self.device, dtype=self.dtype).contiguous()
        if not blocked:
            src = self.pack(src)
        elif src.numel() != self.pop_numel:
            raise ValueError("blocked population tensor must have pop_numel elements")
        self._after_torch()
        check(lib().scd_set_state(self.h, _ptr(src), int(step)))
        self._keep = (src,)

    def save(self, path):
        """Checkpoint to a file: the post-collision state, the step counter,
        the parameters and the solid mask (torch tensors and plain values,
        readable with torch.load(..., weights_only=True))."""
        torch.save({"state": self.get_state().cpu(), "step": int(self.step_count),
                    "params": dict(self.params), "solid": self.solid.cpu()}, path)

    @classmethod
    def load(cls, path, device="cuda", adjoint=False, stream=None):
        """A new lattice resumed from save(): continuing it reproduces the
        uninterrupted run bit for bit."""
        d = torch.load(path, weights_only=True)
        lat = cls(d["params"], d["solid"].numpy(), device=device, adjoint=adjoint, stream=stream)
        lat.set_state(d["state"], d["step"])
        return lat

    def pull_copy(self):
        """One launch of the step's data movement without arithmetic (the
        populations pulled as by a step, stored unchanged in the other
        buffer); the current state is kept."""
        check(lib().scd_pull_copy(self.h))

    def fill_state(self, value):
        check(lib().scd_fill_state(self.h, float(value)))

    def density(self):
        out = torch.empty((2,) + self.shape, dtype=torch.float64, device=self.device)
        self._after_torch()
        check(lib().scd_density(self.h, _ptr(out)))
        self._before_torch()
        return out

    def pressure_tensor(self):
        """(6, nz, ny, nx) FP64: xx, yy, zz, xy, xz, yz (zero at wall nodes)."""
        out = torch.empty((6,) + self.shape, dtype=torch.float64, device=self.device)
        self._after_torch()
        check(lib().scd_pressure_tensor(self.h, _ptr(out)))
        self._before_torch()
        return out

    def surface_tension_z(self, scratch=None):
        """(sum over planes of <P_zz - (P_xx + P_yy)/2>, plane profile)."""
        if scratch is None:
            scratch = torch.empty((6,) + self.shape, dtype=torch.float64, device=self.device)
        g = _D()
        prof = (_D * self.shape[0])()
        self._after_torch()
        check(lib().scd_surface_tension_z(self.h, _ptr(scratch), ctypes.byref(g), prof))
        return g.value, list(prof)

    def radial_tension(self, center, rmax, nbins, scratch=None, periodic=(True, True, True)):
        """(gamma, R_s, profile of P_N - P_T, profile of phi) about center
        (Eq. mechRadGamma); gamma and R_s are NaN without an interface.
        periodic: per axis (x, y, z), whether distances take the minimum
        image (False along an axis bounded by walls)."""
        if scratch is None:
            scratch = torch.empty((6,) + self.shape, dtype=torch.float64, device=self.device)
        c = (_D * 3)(*[float(v) for v in center])
        prof, pphi = (_D * nbins)(), (_D * nbins)()
        rs, g = _D(), _D()
        self._after_torch()
        mask = sum(1 << a for a in range(3) if periodic[a])
        st = lib().scd_radial_tension_axes(self.h, _ptr(scratch), c, mask, float(rmax), int(nbins),
                                           prof, pphi, ctypes.byref(rs), ctypes.byref(g))
        if st not in (SCD_OK, SCD_ENOINTERFACE):
            check(st)
        return g.value, rs.value, list(prof), list(pphi)

    def observables(self, raise_nonfinite=True, raise_drift=True):
        o = ScdObs()
        st = lib().scd_observables(self.h, ctypes.byref(o))
        if (st != SCD_ENONFINITE or raise_nonfinite) and (st != SCD_EDRIFT or raise_drift):
            check(st)
        d = (ctypes.c_double * 2)()
        check(lib().scd_mass_drift(self.h, d))
        return {"mass": (o.mass[0], o.mass[1]), "momentum": tuple(o.momentum), "finite": bool(o.finite),
                "step": o.step, "drift": (d[0], d[1]), "status": st}

    def set_mass_watchdog(self, rel_tol):
        """Flag (SCD_EDRIFT from observables) relative mass drift above
        rel_tol since the state was last set; 0 only measures."""
        check(lib().scd_set_mass_watchdog(self.h, float(rel_tol)))

    def contact_angle(self, cfg, static_scratch=False):
        """Both estimators of Sec. 3; static_scratch: through
        scd_contact_angle_static (scratch in the library's device array)."""
        out = ScdCa()
        c = make_ca_cfg(cfg)
        fn = lib().scd_contact_angle_static if static_scratch else lib().scd_contact_angle
        st = fn(self.h, ctypes.byref(c), ctypes.byref(out))
        if st not in (SCD_OK, SCD_ENOINTERFACE):
            check(st)
        d = {n: getattr(out, n) for n, _ in ScdCa._fields_ if n != "pad"}
        d["status"] = st
        return d

    def ca_seed(self, cfg, dL_dtheta=1.0, out=None, blocked=False):
        b = self.empty_blocked() if (out is None or not blocked) else out
        c = make_ca_cfg(cfg)
        self._after_torch()
        check(lib().scd_ca_seed(self.h, ctypes.byref(c), float(dL_dtheta), _ptr(b)))
        self._before_torch()
        return b if blocked else self.unpack(b, out)

    def adjoint_step(self, state_t, lam_in, lam_out=None, accumulate=False, blocked=False):
        """One reverse step.  accumulate=True adds the parameter gradient to
        the device accumulator (no synchronisation) and returns None for it.
        Population tensors are plain unless blocked=True."""
        if blocked:
            st, li = state_t, lam_in
            lo = torch.zeros_like(lam_in) if lam_out is None else lam_out
        else:
            st, li, lo = self.pack(state_t), self.pack(lam_in), self.empty_blocked()
        self._after_torch()
        dp = None if accumulate else (ctypes.c_double * 5)()
        check(lib().scd_adjoint_step(self.h, _ptr(st), _ptr(li), _ptr(lo), dp))
        self._before_torch()
        if not blocked:
            lo = self.unpack(lo, lam_out)
        return lo, (None if accumulate else list(dp))

    def adjoint_reset(self):
        check(lib().scd_adjoint_reset(self.h))

    def adjoint_read(self):
        g = (ctypes.c_double * 5)()
        check(lib().scd_adjoint_read(self.h, g))
        return list(g)

    def tile(self):
        """(variant index, z-chunk) of the fused step."""
        a, b = _I32(), _I32()
        check(lib().scd_tile_get(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_tile(self, variant, zc):
        check(lib().scd_tile_set(self.h, int(variant), int(zc)))

    def autotune(self, steps_per_trial=10, cache_path=None):
        best = (_I32 * 2)()
        ms = _D()
        cp = cache_path.encode() if cache_path else None
        check(lib().scd_autotune(self.h, int(steps_per_trial), cp, best, ctypes.byref(ms)))
        return tuple(best), ms.value

    def graph_capture(self, nsteps):
        check(lib().scd_graph_capture(self.h, int(nsteps)))

    def graph_replay(self, reps=1):
        check(lib().scd_graph_replay(self.h, int(reps)))


def young_angle(gamma_sg, gamma_sl, gamma_lg):
    """Eq. young in degrees (liquid = droplet species), clamped."""
    return lib().scd_young_angle(float(gamma_sg), float(gamma_sl), float(gamma_lg))


def huang_angle(params, rho_in, rho_out):
    """Huang's estimate (Eq. huangSigmaLG) for droplet species A, degrees."""
    sp = make_params(params)
    return lib().scd_huang_angle(ctypes.byref(sp), float(rho_in), float(rho_out))


def stream_copy(src, dst, stream=None):
    """Copy device tensor src into dst (same byte size, a multiple of 8) with
    the library's STREAM copy kernel on stream; asynchronous."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("source and destination sizes differ")
    check(lib().scd_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream_handle(stream)))


def tile_list():
    """Compiled step variants as (tx, ty, z-march variant, waves per SIMD);
    the list index is the variant index of set_tile."""
    buf = (_I32 * 256)()
    n = _I32()
    check(lib().scd_tile_list(buf, 64, ctypes.byref(n)))
    return [tuple(buf[4 * i:4 * i + 4]) for i in range(n.value)]


def variant_index(tx, ty, zmarch, waves):
    return tile_list().index((tx, ty, zmarch, waves))


class Batch:
    """Many lattices stepped together: one launch per group of members and
    step, cache-blocked in sets (scd_batch_* in include/scdrop.h)."""

    def __init__(self, params_list, solids, device="cuda", stream=None):
        self.device = torch.device(device)
        n = len(params_list)
        arr = (ScdParams * n)(*[make_params(p) for p in params_list])
        nbytes = ctypes.c_size_t()
        check(lib().scd_batch_sizes(n, arr, ctypes.byref(nbytes)))
        self.arena = _alloc_bytes(nbytes.value, self.device).zero_()  # padding slots stay zero
        self.solids = [torch.as_tensor(s, dtype=torch.uint8).to(self.device).contiguous() for s in solids]
        ptrs = (ctypes.c_void_p * n)(*[s.data_ptr() for s in self.solids])
        self.stream = stream
        h = ctypes.c_void_p()
        check(lib().scd_batch_create(n, arr, ptrs, _ptr(self.arena), _stream_handle(stream), ctypes.byref(h)))
        self.h = h
        self.params = [dict(p) for p in params_list]
        self.n = n

    def close(self):
        if getattr(self, "h", None):
            lib().scd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_equilibrium(self, i, rho_a, rho_b):
        ra = _device_f64(rho_a, self.device).reshape(-1)
        rb = _device_f64(rho_b, self.device).reshape(-1)
        torch.cuda.synchronize(self.device)
        check(lib().scd_batch_init_equilibrium(self.h, int(i), _ptr(ra), _ptr(rb)))
        torch.cuda.synchronize(self.device)

    def set_tile(self, variant, zc, grid):
        check(lib().scd_batch_set_tile(self.h, int(variant), int(zc), int(grid)))

    def set_member_tile(self, i, variant, zc):
        check(lib().scd_batch_set_member_tile(self.h, int(i), int(variant), int(zc)))

    def member_tiles(self):
        """[(variant, zc)] of every member."""
        out = []
        for i in range(self.n):
            v, z = _I32(), _I32()
            check(lib().scd_batch_member_tile(self.h, i, ctypes.byref(v), ctypes.byref(z)))
            out.append((v.value, z.value))
        return out

    def set_blocking(self, set_bytes):
        """Step the members in sets of at most set_bytes of state, every step
        of a call on one set before the next (0: one set of all members)."""
        check(lib().scd_batch_set_blocking(self.h, int(set_bytes)))

    def blocking(self):
        """(set_bytes, number of sets)."""
        sb, ns = ctypes.c_int64(), _I32()
        check(lib().scd_batch_blocking(self.h, ctypes.byref(sb), ctypes.byref(ns)))
        return sb.value, ns.value

    def step(self, n=1):
        check(lib().scd_batch_step(self.h, int(n)))

    def autotune(self, steps_per_trial=3, cache_path=None):
        """Fastest (variant, zc, grid) and its ms per step (zc 0: each member
        at its own chunk); members advance."""
        best = (_I32 * 3)()
        ms = _D()
        path = cache_path.encode() if cache_path else None
        check(lib().scd_batch_autotune(self.h, int(steps_per_trial), path, best, ctypes.byref(ms)))
        return tuple(best), ms.value

    def graph_capture(self, nsteps):
        check(lib().scd_batch_graph_capture(self.h, int(nsteps)))

    def graph_replay(self, reps=1):
        check(lib().scd_batch_graph_replay(self.h, int(reps)))

    def view(self, i):
        """(handle, shape, dtype) of member i for observables and state copies."""
        v = ctypes.c_void_p()
        check(lib().scd_batch_lattice(self.h, int(i), ctypes.byref(v)))
        return _View(v, self.params[i], self.device, self.stream)


class _View(Lattice):
    """Lattice interface over a batch member (buffers owned by the batch)."""

    def __init__(self, h, params, device, stream):  # noqa: D401 - no buffers of its own
        self.h = h
        self.stream = stream
        self.params = dict(params)
        self.device = device
        self.sp = make_params(params)
        self.shape = (params["nz"], params["ny"], params["nx"])
        self.N = params["nx"] * params["ny"] * params["nz"]
        self.dtype = _torch_dtype(self.sp)
        pop_b = ctypes.c_size_t()
        check(lib().scd_sizes(ctypes.byref(self.sp), ctypes.byref(pop_b), None))
        self.pop_numel = pop_b.value // torch.empty((), dtype=self.dtype).element_size()

    def close(self):
        self.h = None  # owned by the batch
