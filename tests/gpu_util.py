"""Helpers shared by the GPU parity tests (comparison only, no method arithmetic)."""
import numpy as np

TWO_PI = 2 * np.pi


def circ(a, b):
    """Circular distance between angle arrays (radians)."""
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) % TWO_PI
    return np.minimum(d, TWO_PI - d)


def colour_mask(L, c):
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    return (((x + y + z) & 1) == c).ravel()


def field_numpy(theta, L):
    """Neighbour field h = sum of the six neighbouring unit vectors (numpy rolls)."""
    g = np.asarray(theta, dtype=np.float64).reshape(L, L, L)
    hx = sum(np.cos(np.roll(g, s, axis=a)) for a in range(3) for s in (1, -1)).ravel()
    hy = sum(np.sin(np.roll(g, s, axis=a)) for a in range(3) for s in (1, -1)).ravel()
    return hx, hy


def gpu_states(sim, lattice=0):
    return np.stack([sim.get_angles(lattice, k) for k in range(sim.R[lattice])])
