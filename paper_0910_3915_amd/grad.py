"""torch.autograd.Function over the library's checkpointed adjoint driver.

Forward: scd_ckpt_forward runs the lattice from the initial densities,
storing the state every ``ckpt_every`` steps, and returns the loss
(theta_E2 - target)^2 in deg^2.  Backward: scd_ckpt_backward recomputes each
segment from its checkpoint and runs the hand-written adjoint steps in
reverse, giving dL/d(rho_wall_A, rho_wall_B, g_ab, g_wall_A, g_wall_B).
"""
import ctypes

import torch

from . import binding as B


class GradSetup:
    """Buffers and settings of one differentiable run (caller keeps it alive).

    ckpt_every = K stores a state every K steps and recomputes each segment
    (one level).  With inner = K2 < K the backward pass also checkpoints
    every K2 steps inside a segment (two levels), for lattices whose states
    are too large to hold K of them.  rho_a = rho_b = None starts every
    forward pass from the lattice's current state instead of re-initialising.
    moment_cache keeps the densities and momenta of the post-stream
    populations of each recomputed segment (8 x N reals per step of a
    segment), which spares the adjoint its own pass over the populations to
    form them; the gradient is the same bit for bit.
    """

    def __init__(self, params, solid, rho_a, rho_b, nsteps, ckpt_every, ca_cfg, target_deg,
                 device="cuda", stream=None, inner=None, lattice=None, moment_cache=True):
        self.lat = lattice or B.Lattice(params, solid, device=device, adjoint=True, stream=stream)
        self.params = dict(params)
        self.nsteps = int(nsteps)
        self.K = int(ckpt_every)
        self.K2 = int(inner) if inner else None
        self.cfg = B.make_ca_cfg(ca_cfg)
        self.target = float(target_deg)
        dev = self.lat.device
        self.rho_a = None if rho_a is None else B._device_f64(rho_a, dev).reshape(-1)
        self.rho_b = None if rho_b is None else B._device_f64(rho_b, dev).reshape(-1)
        nseg = (self.nsteps + self.K - 1) // self.K
        shape = (self.lat.pop_numel,)  # one population buffer (blocked layout)
        dt = self.lat.dtype
        self.ckpt = torch.empty((nseg,) + shape, dtype=dt, device=dev)
        if self.K2:
            self.mid = torch.empty(((self.K + self.K2 - 1) // self.K2,) + shape, dtype=dt, device=dev)
        self.lam = torch.empty((2,) + shape, dtype=dt, device=dev)
        self.seg_len = self.K2 or self.K
        self.mom_cache = None
        if moment_cache and self.seg_len > 1:
            self.mom_cache = torch.empty((self.seg_len - 1, 8) + self.lat.shape, dtype=dt, device=dev)
        # recomputed states of one segment: sized at each backward pass for
        # the step variant then in use (two buffers when the moment cache
        # serves the adjoint, else one per recomputed step)
        self.seg = torch.empty((0,) + shape, dtype=dt, device=dev)
        self.theta = float("nan")
        self.start = None if rho_a is not None else self.lat.get_state()

    def apply_params(self, values):
        v = [float(x) for x in values]
        p = dict(self.params, rho_wall=(v[0], v[1]), g_ab=v[2], g_wall=(v[3], v[4]))
        self.lat.set_params(p)
        self.params = p

    def forward(self):
        self.lat._after_torch()
        out = (ctypes.c_double * 2)()
        if self.rho_a is None:
            # every pass starts from the same stored state
            self.lat.set_state(self.start, self.lat.step_count)
            ra = rb = None
        else:
            ra, rb = B._ptr(self.rho_a), B._ptr(self.rho_b)
        B.check(B.lib().scd_ckpt_forward(self.lat.h, ra, rb, self.nsteps, self.K, B._ptr(self.ckpt),
                                         ctypes.byref(self.cfg), self.target, out))
        self.theta = out[1]
        return out[0]

    def backward(self):
        g = (ctypes.c_double * 5)()
        # the cache is registered for this sweep only, so the lattice never
        # keeps a pointer to a buffer this object may outlive
        if self.mom_cache is not None:
            B.check(B.lib().scd_ckpt_moment_cache(self.lat.h, B._ptr(self.mom_cache),
                                                  self.mom_cache.shape[0]))
        try:
            self._sweep(g)
        finally:
            if self.mom_cache is not None:
                B.check(B.lib().scd_ckpt_moment_cache(self.lat.h, None, 0))
        return list(g)

    def _sweep(self, g):
        n = ctypes.c_int64()
        B.check(B.lib().scd_ckpt_seg_states(self.lat.h, self.seg_len, ctypes.byref(n)))
        need = max(n.value, 1)
        if self.seg.shape[0] != need:
            self.seg = None
            self.seg = torch.empty((need, self.lat.pop_numel), dtype=self.lat.dtype, device=self.lat.device)
        if self.K2:
            B.check(B.lib().scd_ckpt_backward2(self.lat.h, self.nsteps, self.K, self.K2, B._ptr(self.ckpt),
                                               B._ptr(self.mid), B._ptr(self.seg), B._ptr(self.lam),
                                               ctypes.byref(self.cfg), self.target, g))
        else:
            B.check(B.lib().scd_ckpt_backward(self.lat.h, self.nsteps, self.K, B._ptr(self.ckpt),
                                              B._ptr(self.seg), B._ptr(self.lam), ctypes.byref(self.cfg),
                                              self.target, g))


class ContactAngleFn(torch.autograd.Function):
    """loss = ContactAngleFn.apply(wall, setup) with wall = tensor of
    (rho_wall_A, rho_wall_B, g_ab, g_wall_A, g_wall_B) (float64, CPU)."""

    @staticmethod
    def forward(ctx, wall, setup):
        setup.apply_params(wall.detach().cpu().tolist())
        loss = setup.forward()
        ctx.setup = setup
        return torch.tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.setup.backward()
        return grad_out * torch.tensor(g, dtype=torch.float64), None
