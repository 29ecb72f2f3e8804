"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  Nothing here computes any part of the lattice Boltzmann method: it
only builds parameter sets, solid masks and initial density fields.

Initial state (Sec. 2 of the paper): a spherical cap of component A on a
smooth wall, surrounded by component B.  Inside the cap (rho_A, rho_B) =
(rho_in, rho_out), outside the values are swapped, plus i.i.d. uniform noise
of amplitude ``noise`` drawn with ``numpy.random.default_rng(seed)``: first
the A noise field, then the B noise field, each in x-fastest order over the
whole box (values at solid nodes are drawn and then ignored).
"""
import numpy as np

DEFAULT_TAU = (1.0, 1.0)


def params(nx, ny, nz, g_ab, rho_wall=(0.5, 0.5), g_wall=None, tau=DEFAULT_TAU,
           psi=0, w_axis=1.0, w_diag=1.0, dtype="f64"):
    """Parameter dict understood by both the oracle wrapper and the GPU binding.

    ``g_wall`` defaults to ``g_ab`` for both species (one coupling for
    fluid-fluid and fluid-wall interaction, as in the paper's runs).
    """
    if g_wall is None:
        g_wall = (g_ab, g_ab)
    return {"nx": int(nx), "ny": int(ny), "nz": int(nz), "psi": int(psi),
            "tau": (float(tau[0]), float(tau[1])), "g_ab": float(g_ab),
            "g_wall": (float(g_wall[0]), float(g_wall[1])),
            "rho_wall": (float(rho_wall[0]), float(rho_wall[1])),
            "w_axis": float(w_axis), "w_diag": float(w_diag), "dtype": dtype}


def asymmetric_wall(delta, mean=0.5):
    """Wall content (rho_wall_A, rho_wall_B) with difference ``delta``."""
    return (mean + delta / 2.0, mean - delta / 2.0)


def walls_mask(nx, ny, nz, floor=True, ceiling=True):
    """Solid layers at z = 0 and z = nz - 1; periodic in x and y."""
    m = np.zeros((nz, ny, nx), np.uint8)
    if floor:
        m[0] = 1
    if ceiling:
        m[nz - 1] = 1
    return m


def posts_mask(nx, ny, nz, width=6, pitch=12, height=12):
    """Floor, ceiling and a square array of posts on the floor:
    solid where x mod pitch < width and y mod pitch < width, 1 <= z <= height."""
    m = walls_mask(nx, ny, nz)
    x = np.arange(nx)[None, :] % pitch < width
    y = np.arange(ny)[:, None] % pitch < width
    post = (x & y).astype(np.uint8)
    m[1:height + 1] |= post[None, :, :]
    return m


def cap_densities(nx, ny, nz, radius, z_wall, solid, rho_in=0.7, rho_out=0.04,
                  noise=1e-3, seed=0, center=None):
    """Spherical cap of A centred at (nx/2, ny/2, z_wall) (or ``center``)."""
    if center is None:
        center = (nx / 2.0, ny / 2.0, z_wall)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2
    inside = (r2 <= radius * radius) & (z > z_wall)
    rho_a = np.where(inside, rho_in, rho_out).astype(np.float64)
    rho_b = np.where(inside, rho_out, rho_in).astype(np.float64)
    if noise:
        rng = np.random.default_rng(seed)
        rho_a = rho_a + rng.uniform(-noise, noise, size=rho_a.shape)
        rho_b = rho_b + rng.uniform(-noise, noise, size=rho_b.shape)
    solid = np.asarray(solid).astype(bool)
    rho_a[solid] = 0.0
    rho_b[solid] = 0.0
    return rho_a, rho_b


def cube_densities(nx, ny, nz, side, z_wall, solid, rho_in=0.7, rho_out=0.04, noise=1e-3, seed=0):
    """A cube of A with edge ``side`` standing on the wall top z_wall,
    centred on the column (nx/2, ny/2): nodes with |x - nx/2| < side/2,
    |y - ny/2| < side/2 and z_wall < z <= z_wall + side."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    h = side / 2.0
    inside = (np.abs(x - nx / 2.0) < h) & (np.abs(y - ny / 2.0) < h) & (z > z_wall) & (z <= z_wall + side)
    rho_a = np.where(inside, rho_in, rho_out).astype(np.float64)
    rho_b = np.where(inside, rho_out, rho_in).astype(np.float64)
    if noise:
        rng = np.random.default_rng(seed)
        rho_a = rho_a + rng.uniform(-noise, noise, size=rho_a.shape)
        rho_b = rho_b + rng.uniform(-noise, noise, size=rho_b.shape)
    solid = np.asarray(solid).astype(bool)
    rho_a[solid] = 0.0
    rho_b[solid] = 0.0
    return rho_a, rho_b


def sphere_densities(n, radius, rho_in=0.7, rho_out=0.04, center=None):
    """Free droplet of A in a fully periodic cube (no walls)."""
    if center is None:
        center = (n / 2.0, n / 2.0, n / 2.0)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r2 = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2
    inside = r2 <= radius * radius
    rho_a = np.where(inside, rho_in, rho_out).astype(np.float64)
    rho_b = np.where(inside, rho_out, rho_in).astype(np.float64)
    return rho_a, rho_b


def uniform_noise_densities(shape, rho_a, rho_b, noise, seed=0):
    rng = np.random.default_rng(seed)
    ra = rho_a + rng.uniform(-noise, noise, size=shape)
    rb = rho_b + rng.uniform(-noise, noise, size=shape)
    return ra, rb


def ca_cfg(nx, ny, z_solid_top=0, offset=5, eps=0.2):
    """Contact-angle measurement: column through the placement centre."""
    return {"ic": nx // 2, "jc": ny // 2, "z_solid_top": int(z_solid_top),
            "offset": int(offset), "eps": float(eps)}


# ---------------------------------------------------------------- workloads
def droplet_case(nx, ny, nz, radius, g_ab, delta=0.0, seed=0, dtype="f64", noise=1e-3,
                 offset=5, mask=None, z_solid_top=0):
    """Droplet on the floor of a box with walls at z = 0 and z = nz - 1."""
    solid = walls_mask(nx, ny, nz) if mask is None else mask
    p = params(nx, ny, nz, g_ab, rho_wall=asymmetric_wall(delta), dtype=dtype)
    z_wall = z_solid_top + 0.5
    ra, rb = cap_densities(nx, ny, nz, radius, z_wall, solid, noise=noise, seed=seed)
    return {"params": p, "solid": solid, "rho_a": ra, "rho_b": rb,
            "ca": ca_cfg(nx, ny, z_solid_top, offset)}


def config_small_fp64(seed=0):
    """32^3, walls at z = 0 and 31, cap radius 8, g_ab = g_wall = 0.1,
    rho_wall = (0.5, 0.5), tau = 1, psi = rho; 1000 steps."""
    return droplet_case(32, 32, 32, 8.0, 0.1, 0.0, seed=seed)


def config_throughput(delta=0.0, dtype="f64", seed=0):
    """128 x 128 x 64, cap radius 24, g_ab = g_wall = 0.12; 20000 steps."""
    return droplet_case(128, 128, 64, 24.0, 0.12, delta, seed=seed, dtype=dtype)


def config_throughput_twin(delta=0.0, seed=0):
    """Half-size twin: 64 x 64 x 32, cap radius 12."""
    return droplet_case(64, 64, 32, 12.0, 0.12, delta, seed=seed)


THROUGHPUT_DELTAS = tuple(np.round(np.linspace(-0.4, 0.4, 9), 10))


def config_gradient(dtype="f64", seed=0):
    """64 x 64 x 48, cap radius 14, g_ab = g_wall = 0.12, rho_wall = (0.5, 0.5)."""
    return droplet_case(64, 64, 48, 14.0, 0.12, 0.0, seed=seed, dtype=dtype)


def config_gradient_tiny(seed=0):
    """16 x 16 x 12, cap radius 5, reference offset 2 (adjoint check box)."""
    return droplet_case(16, 16, 12, 5.0, 0.12, 0.0, seed=seed, offset=2)


def config_posts(seed=0, dtype="f32"):
    """384 x 384 x 192 with square posts (width 6, pitch 12, height 12),
    cap radius 80 resting on the post tops (Cassie start: gaps hold B),
    wall asymmetry -0.3, g_ab = 0.12."""
    nx, ny, nz = 384, 384, 192
    solid = posts_mask(nx, ny, nz)
    p = params(nx, ny, nz, 0.12, rho_wall=asymmetric_wall(-0.3), dtype=dtype)
    ra, rb = cap_densities(nx, ny, nz, 80.0, 12.5, solid, seed=seed)
    return {"params": p, "solid": solid, "rho_a": ra, "rho_b": rb,
            "ca": ca_cfg(nx, ny, z_solid_top=12, offset=5)}


def planar_case(kind, g_ab, rho_wall=(0.5, 0.5), nx=32, ny=8, nz=128, dtype="f64",
                rho_in=0.7, rho_out=0.04):
    """Planar systems of the surface-tension measurement, periodic on all
    axes, interfaces normal to z:
      "AB": an A lamella on z in [nz/4, 3nz/4) in B (two A-B interfaces);
      "Aw"/"Bw": solid on z < nz/2, the upper half filled with the A-rich
      (B-rich) phase (two fluid-wall interfaces).
    The A-rich phase holds (rho_in, rho_out), the B-rich phase the reverse;
    g_wall = g_ab."""
    z = np.arange(nz)[:, None, None] * np.ones((1, ny, nx))
    solid = np.zeros((nz, ny, nx), np.uint8)
    if kind == "AB":
        a_rich = (z >= nz // 4) & (z < 3 * nz // 4)
    else:
        solid[: nz // 2] = 1
        a_rich = np.full(z.shape, kind == "Aw")
    ra = np.where(a_rich, rho_in, rho_out).astype(np.float64)
    rb = np.where(a_rich, rho_out, rho_in).astype(np.float64)
    ra[solid == 1] = 0.0
    rb[solid == 1] = 0.0
    p = params(nx, ny, nz, g_ab, rho_wall=tuple(rho_wall), dtype=dtype)
    return {"params": p, "solid": solid, "rho_a": ra, "rho_b": rb, "kind": kind}


def batch_draw(n=64, seed=0):
    """Box sizes and parameters of the batched sweep: Lx, Ly uniform in
    {64..128}, Lz in {48..96}, all multiples of 8; g_ab uniform in
    [0.08, 0.16]; wall asymmetry uniform in [-0.4, 0.4]; radius 0.2 min(Lx, Ly)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        lx = 8 * int(rng.integers(8, 17))
        ly = 8 * int(rng.integers(8, 17))
        lz = 8 * int(rng.integers(6, 13))
        g = float(rng.uniform(0.08, 0.16))
        d = float(rng.uniform(-0.4, 0.4))
        out.append({"nx": lx, "ny": ly, "nz": lz, "g_ab": g, "delta": d,
                    "radius": 0.2 * min(lx, ly)})
    return out
