"""Shared helpers of the GPU tests (the HIP library against the oracle)."""
import numpy as np
import torch

import oracle as O


def gpu_density(L):
    """(nz, ny, nx, 2) FP64 numpy densities of a GPU lattice."""
    return np.moveaxis(L.density().cpu().numpy(), 0, -1)


def gpu_state_as_oracle(L):
    """A GPU lattice's state in the oracle's array order, to compare with an
    oracle result (never to feed the oracle)."""
    return O.from_gpu_layout(L.get_state().double().cpu().numpy())


def oracle_run(case, steps, params=None):
    Lo = O.Lattice(params or case["params"], case["solid"])
    Lo.init_equilibrium(case["rho_a"], case["rho_b"])
    Lo.step(steps)
    return Lo


def announce(msg):
    print(msg, flush=True)


def sync():
    torch.cuda.synchronize()
