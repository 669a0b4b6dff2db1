"""Seeded media and sources (stand-ins for the paper's workloads, Sec. 5).

The paper's 2D heterogeneous models (Sec. 5.4: "linear" and "wedge") and the 3D
Overthrust model (Sec. 5.5) are not available; these generators produce media of
the same kind: horizontal layered slowness with smooth noise in 2D, a
depth-increasing velocity with dipping layers and a fast ellipsoidal inclusion in
3D.  Arrays have shape n[::-1] (x fastest), float64.
"""
import numpy as np
from scipy.ndimage import gaussian_filter


def omega_for_ppw(h, ppw=10.0, kappa_max=1.0):
    """Angular frequency giving `ppw` grid points per shortest wavelength.

    Wavelength = 2 pi / (omega kappa); the shortest one sits where kappa is largest.
    """
    return 2.0 * np.pi / (ppw * h * kappa_max)


def homogeneous(n, value=1.0):
    return np.full(tuple(reversed(n)), float(value))


def linear_kappa2(n, lo=0.25, hi=1.0):
    """kappa^2 varying linearly with depth (last axis) from lo to hi (Sec. 5.4)."""
    shape = tuple(reversed(n))
    depth = np.linspace(0.0, 1.0, n[-1])
    k2 = lo + (hi - lo) * depth
    k = np.sqrt(k2)
    return np.broadcast_to(k.reshape((n[-1],) + (1,) * (len(n) - 1)), shape).copy()


def layered_2d(n, seed, layers=(8, 14), kappa_range=(0.25, 1.0), noise=0.05,
               sigma_cells=8.0):
    """Horizontal layers (depth = y) with per-layer kappa ~ U[kappa_range] plus
    Gaussian-smoothed noise scaled to max |xi| = 1, kappa <- kappa (1 + noise xi)."""
    rng = np.random.default_rng(seed)
    nx, ny = n
    L = int(rng.integers(layers[0], layers[1] + 1))
    cuts = np.unique(rng.integers(1, ny, size=L - 1))
    kl = rng.uniform(kappa_range[0], kappa_range[1], size=len(cuts) + 1)
    layer_of_row = np.searchsorted(cuts, np.arange(ny), side="right")
    kappa = np.repeat(kl[layer_of_row][:, None], nx, axis=1)
    xi = gaussian_filter(rng.standard_normal((ny, nx)), sigma_cells, mode="reflect")
    xi /= np.max(np.abs(xi))
    return kappa * (1.0 + noise * xi)


def geophysical_3d(n, seed, v_range=(1.5, 4.5), layers=(4, 8), v_inclusion=5.0,
                   v_ref=1.5):
    """3D velocity increasing with depth (z) over random dipping planar layers and
    one rotated ellipsoid at v_inclusion; returns kappa = v_ref / v."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.linspace(0, 1, nz), np.linspace(0, 1, ny),
                          np.linspace(0, 1, nx), indexing="ij")
    L = int(rng.integers(layers[0], layers[1] + 1))
    depths = np.sort(rng.uniform(0.05, 0.95, size=L - 1))
    vel = np.sort(rng.uniform(v_range[0], v_range[1], size=L))
    vel[0], vel[-1] = v_range[0], v_range[1]
    v = np.full(z.shape, vel[0])
    for i, d0 in enumerate(depths):
        dip = np.deg2rad(rng.uniform(0.0, 20.0))
        az = rng.uniform(0.0, 2 * np.pi)
        surface = d0 + np.tan(dip) * ((x - 0.5) * np.cos(az) + (y - 0.5) * np.sin(az))
        v = np.where(z >= surface, vel[i + 1], v)
    c = rng.uniform(1 / 3, 2 / 3, size=3)
    ax = rng.uniform(0.08, 0.2, size=3)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    p = np.stack([x - c[0], y - c[1], z - c[2]], axis=-1) @ q
    inside = np.sum((p / ax) ** 2, axis=-1) <= 1.0
    v = np.where(inside, v_inclusion, v)
    return v_ref / v


def point_source(n, where=None):
    """Unit point source at the centre node (Sec. 5: 'a point source in the centre')."""
    q = np.zeros(tuple(reversed(n)), dtype=complex)
    if where is None:
        where = tuple(k // 2 for k in n)
    q[tuple(reversed(where))] = 1.0
    return q


def random_sources(n, count, seed, margin):
    """`count` unit point sources at distinct random nodes at least `margin` nodes
    away from every face; returns (count, N) complex array."""
    rng = np.random.default_rng(seed)
    N = int(np.prod(n))
    out = np.zeros((count, N), dtype=complex)
    for s in range(count):
        pos = [int(rng.integers(margin, k - margin)) for k in n]
        lin = 0
        stride = 1
        for d, p in enumerate(pos):
            lin += p * stride
            stride *= n[d]
        out[s, lin] = 1.0
    return out
