"""Python face of the XY-model hot path: a thin wrapper over the C ABI.

PyTorch only provides device memory (the angle buffer and observable rings)
and the stream; all Monte Carlo work happens in libxy.so's HIP kernels.
"""
import ctypes

import numpy as np

from . import _capi as C


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Sim:
    """A batch of periodic L^3 XY lattices, each with a beta-ladder of replicas.

    Parameters mirror xy_config: ``L`` (list of even sizes), ``betas`` (list of
    ascending ladders, one per lattice), ``seed``, ``prec`` ('fp32'|'fp64'),
    ``start`` ('random'|'ordered'), ``recheck`` (FP32 near-threshold float64
    re-decision), ``stream`` (a torch.cuda.Stream or None for the current one).
    """

    def __init__(self, L, betas, seed=1, prec="fp32", start="random", recheck=True,
                 fused_or=True, stream=None, device=None):
        import torch
        self.L = [int(v) for v in (L if isinstance(L, (list, tuple)) else [L])]
        if betas and np.ndim(betas[0]) == 0:
            betas = [betas]
        self.betas = [np.ascontiguousarray(b, dtype=np.float64) for b in betas]
        if len(self.betas) != len(self.L):
            raise ValueError("one beta ladder per lattice")
        self.R = [len(b) for b in self.betas]
        self.R_total = sum(self.R)
        self.pos_base = np.concatenate([[0], np.cumsum(self.R)[:-1]]).astype(int).tolist()
        self.seed = int(seed)
        self.prec = {"fp32": C.XY_FP32, "fp64": C.XY_FP64}[prec]
        self._Larr = (ctypes.c_int32 * len(self.L))(*self.L)
        self._Rarr = (ctypes.c_int32 * len(self.R))(*self.R)
        self._beta = np.ascontiguousarray(np.concatenate(self.betas))
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        cfg = C.XYConfig()
        cfg.n_lattices = len(self.L)
        cfg.L = self._Larr
        cfg.n_replicas = self._Rarr
        cfg.beta = self._beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        cfg.seed = self.seed
        cfg.prec = self.prec
        cfg.start = {"random": C.XY_START_RANDOM, "ordered": C.XY_START_ORDERED}[start]
        cfg.flags = (0 if recheck else C.XY_F_NO_RECHECK) | (0 if fused_or else C.XY_F_NO_FUSED_OR)
        nbytes = C.lib().xy_angles_bytes(ctypes.byref(cfg))
        if nbytes == 0:
            C.check(C.lib().xy_init(ctypes.byref(cfg), ctypes.byref(ctypes.c_void_p())))
        # caller-owned angle storage (torch), adopted by the library
        self.angles = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        cfg.angles_dev = ctypes.c_void_p(self.angles.data_ptr())
        cfg.stream = _stream_handle(self.stream)
        self._cfg = cfg
        ctx = ctypes.c_void_p()
        C.check(C.lib().xy_init(ctypes.byref(cfg), ctypes.byref(ctx)))
        self._ctx = ctx

    # -- verbs ---------------------------------------------------------------
    def sweep(self, n_metro=1, n_or=1):
        C.check(C.lib().xy_sweep(self._ctx, int(n_metro), int(n_or)), self._ctx)

    def measure(self, out=None):
        """Observables (R_total, 5) = (E, e, |m|, m^2, m^4) by position index.

        With ``out`` a float64 CUDA tensor of that shape the call stays on the
        device and returns ``out``; otherwise a numpy array is returned."""
        if out is not None:
            self._check_ring("out", out, self.R_total * 5)
            C.check(C.lib().xy_measure(self._ctx, ctypes.c_void_p(out.data_ptr()), 1), self._ctx)
            return out
        obs = np.zeros((self.R_total, 5), dtype=np.float64)
        C.check(C.lib().xy_measure(self._ctx, obs.ctypes.data_as(ctypes.c_void_p), 0), self._ctx)
        return obs

    def exchange(self, with_counts=False):
        if with_counts:
            acc = np.zeros(self.R_total, dtype=np.int64)
            C.check(C.lib().xy_exchange(self._ctx, acc.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), self._ctx)
            return acc
        C.check(C.lib().xy_exchange(self._ctx, None), self._ctx)
        return None

    def run(self, n_sweeps, n_metro=1, n_or=1, exchange_every=1, obs=None, bonds=None):
        """Graph-replayed loop.  ``obs`` (optional) is a float64 tensor of
        shape (n_sweeps, R_total, 5) receiving every sweep's observables;
        ``bonds`` (optional) one of shape (n_sweeps, R_total, 6) receiving the
        bond sums (C_x, C_y, C_z, I_x, I_y, I_z) of Eq. (6).  Either may live
        on the GPU or in pinned host memory (``pin_memory=True``), which the
        kernels write directly."""
        self._check_ring("obs", obs, n_sweeps * self.R_total * 5)
        self._check_ring("bonds", bonds, n_sweeps * self.R_total * 6)
        ptr = ctypes.c_void_p(obs.data_ptr()) if obs is not None else None
        bptr = ctypes.c_void_p(bonds.data_ptr()) if bonds is not None else None
        C.check(C.lib().xy_run_ex(self._ctx, int(n_sweeps), int(n_metro), int(n_or),
                                  int(exchange_every), ptr, bptr), self._ctx)

    def _check_ring(self, name, t, n):
        """The kernels write n float64 values through the ring's pointer."""
        if t is None:
            return
        import torch
        reachable = t.device.type == "cuda" or (t.device.type == "cpu" and t.is_pinned())
        if t.dtype != torch.float64 or not reachable or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor on the GPU or in pinned host memory")
        if t.numel() < n:
            raise ValueError(f"{name} holds {t.numel()} values, the run writes {n}")

    def bond_sums(self):
        """(R_total, 6) bond sums C_x, C_y, C_z, I_x, I_y, I_z of the current state."""
        out = np.zeros((self.R_total, 6), dtype=np.float64)
        C.check(C.lib().xy_get_bond_sums(self._ctx, out.ctypes.data_as(ctypes.c_void_p), 0), self._ctx)
        return out

    def sweep_profiled(self, n_metro=1, n_or=1):
        """xy_sweep with HIP events around each group of consecutive launches of
        one kind: returns the group's milliseconds and its launch count, keyed
        'metro' (half-sweeps, float64 re-decision included), 'over'
        (half-sweeps), 'over_fused' (fused substeps) and 'other'."""
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_int32 * 4)()
        C.check(C.lib().xy_sweep_profiled(self._ctx, int(n_metro), int(n_or), ms, n), self._ctx)
        keys = ("metro", "over", "over_fused", "other")
        return dict(zip(keys, list(ms))), dict(zip(keys, list(n)))

    def autotune(self, n_metro=1, n_or=1, reps=3):
        """Time the admissible tilings of every lattice and keep the fastest
        (the chain state is saved and restored around the timing)."""
        C.check(C.lib().xy_autotune(self._ctx, int(n_metro), int(n_or), int(reps)), self._ctx)
        return [self.get_tiling(l) for l in range(len(self.L))]

    def set_tiling(self, lattice, ty, tz, grid_cap=0):
        C.check(C.lib().xy_set_tiling(self._ctx, int(lattice), int(ty), int(tz), int(grid_cap)), self._ctx)

    def set_proposal_window(self, window):
        """0: uniform Metropolis proposal; 0 < window <= 2 pi: theta + window (U - 1/2)."""
        C.check(C.lib().xy_set_proposal_window(self._ctx, float(window)), self._ctx)

    def set_tiling_fused(self, lattice, ty, tz):
        C.check(C.lib().xy_set_tiling_fused(self._ctx, int(lattice), int(ty), int(tz)), self._ctx)

    def get_tiling_fused(self, lattice=0):
        ty, tz = ctypes.c_int32(), ctypes.c_int32()
        C.check(C.lib().xy_get_tiling_fused(self._ctx, int(lattice), ctypes.byref(ty), ctypes.byref(tz)), self._ctx)
        return ty.value, tz.value

    def get_tiling(self, lattice=0):
        ty, tz, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        C.check(C.lib().xy_get_tiling(self._ctx, int(lattice), ctypes.byref(ty), ctypes.byref(tz),
                                      ctypes.byref(g)), self._ctx)
        return ty.value, tz.value, g.value

    # -- state ----------------------------------------------------------------
    def get_angles(self, lattice=0, beta_pos=0):
        n = self.L[lattice] ** 3
        out = np.empty(n, dtype=np.float64)
        C.check(C.lib().xy_get_angles(self._ctx, lattice, beta_pos,
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._ctx)
        return out

    def get_angles_fused_mid(self, lattice=0, beta_pos=0):
        """The fused over-relaxation pass's second buffer: after a sweep with
        2m fused substeps, the configuration after the one before the last."""
        n = self.L[lattice] ** 3
        out = np.empty(n, dtype=np.float64)
        C.check(C.lib().xy_get_angles_fused_mid(self._ctx, lattice, beta_pos,
                                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._ctx)
        return out

    def get_sites(self, sites, lattice=0, beta_pos=0):
        """Angles (radians) of the given natural site indices."""
        idx = np.ascontiguousarray(sites, dtype=np.int64)
        out = np.empty(idx.size, dtype=np.float64)
        C.check(C.lib().xy_get_sites(self._ctx, lattice, beta_pos, idx.size,
                                     idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._ctx)
        return out

    def set_angles(self, theta, lattice=0, beta_pos=0):
        a = np.ascontiguousarray(theta, dtype=np.float64)
        if a.size != self.L[lattice] ** 3:
            raise ValueError(f"expected {self.L[lattice] ** 3} angles, got {a.size}")
        C.check(C.lib().xy_set_angles(self._ctx, lattice, beta_pos,
                                      a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._ctx)

    def counters(self):
        t, tau = ctypes.c_uint64(), ctypes.c_uint64()
        C.check(C.lib().xy_get_counters(self._ctx, ctypes.byref(t), ctypes.byref(tau)), self._ctx)
        return t.value, tau.value

    def permutation(self, lattice=0):
        out = (ctypes.c_int32 * self.R[lattice])()
        C.check(C.lib().xy_get_permutation(self._ctx, lattice, out), self._ctx)
        return list(out)

    def metro_accepts(self):
        acc = np.zeros(self.R_total, dtype=np.int64)
        C.check(C.lib().xy_get_metro_accepts(self._ctx, acc.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), self._ctx)
        return acc

    def recheck_overflow(self):
        """Near-threshold Metropolis decisions that did not fit the float64
        re-decision queue since the context was created (they kept their
        float32 decision)."""
        n = ctypes.c_uint64()
        C.check(C.lib().xy_get_recheck_overflow(self._ctx, ctypes.byref(n)), self._ctx)
        return n.value

    def swap_accepts(self):
        """Cumulative accepted exchanges of pair (p, p+1) per position index."""
        acc = np.zeros(self.R_total, dtype=np.int64)
        C.check(C.lib().xy_get_swap_accepts(self._ctx, acc.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), self._ctx)
        return acc

    def get_state(self):
        size = ctypes.c_size_t()
        C.check(C.lib().xy_get_state(self._ctx, None, ctypes.byref(size)), self._ctx)
        buf = ctypes.create_string_buffer(size.value)
        C.check(C.lib().xy_get_state(self._ctx, buf, ctypes.byref(size)), self._ctx)
        return bytes(buf.raw[: size.value])

    def set_state(self, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        C.check(C.lib().xy_set_state(self._ctx, buf, len(blob)), self._ctx)

    def close(self):
        if getattr(self, "_ctx", None):
            C.lib().xy_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
