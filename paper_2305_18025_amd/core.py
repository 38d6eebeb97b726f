"""Python front end of libpimdb: device buffers and streams from PyTorch,
every computation in the HIP library.

Positions, forces and velocities are float64 CUDA tensors holding the packed
bead-major SoA layout of the C ABI: system s occupies ``3 * P_s * N_s``
consecutive elements starting at ``offsets[s]``, viewed as ``(P_s, 3, N_s)``.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check


def _as_list(x, S, name, typ):
    if np.ndim(x) == 0:
        return [typ(x)] * S
    x = list(x)
    if len(x) != S:
        raise ValueError("%s has %d entries, expected %d" % (name, len(x), S))
    return [typ(v) for v in x]


class BosonicExchange:
    """Exchange potential V^[1,N] and bead forces for a batch of systems on one GPU.

    Parameters may be scalars (one system, or shared by the batch) or
    sequences of length S.  ``omega_p`` defaults to sqrt(P)/beta (hbar = 1).
    """

    def __init__(self, N, P, beta, m=1.0, omega_p=None, *, device=0, box=0.0, trap=0.0,
                 precision="fp64", threads=0, per_thread=0, split=-1, algorithm="fast", shift="min",
                 pair=None):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("BosonicExchange needs a GPU")
        S = 1 if np.ndim(N) == 0 else len(N)
        self.S = S
        self.N = _as_list(N, S, "N", int)
        self.P = _as_list(P, S, "P", int)
        self.beta = _as_list(beta, S, "beta", float)
        self.m = _as_list(m, S, "m", float)
        if omega_p is None:
            self.omega_p = [float(np.sqrt(p) / b) for p, b in zip(self.P, self.beta)]
        else:
            self.omega_p = _as_list(omega_p, S, "omega_p", float)
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self._captured = False
        self._old_workspaces = []
        h = ctypes.c_void_p()
        st = torch.cuda.current_stream(self.device).cuda_stream
        check(self.lib.pimdb_create(ctypes.byref(h), self.device.index or 0, ctypes.c_void_p(st)))
        self._h = h
        self.box = float(box)
        self.trap = float(trap)
        self.precision = precision
        check(self.lib.pimdb_set_box(h, self.box), h)
        check(self.lib.pimdb_set_trap(h, self.trap), h)
        mode = {"fp64": _lib.PIMDB_FP64, "mixed": _lib.PIMDB_MIXED, "fp64_direct": _lib.PIMDB_FP64_DIRECT}[precision]
        check(self.lib.pimdb_set_precision(h, mode), h)
        arr = lambda t, v: (t * S)(*v)
        check(self.lib.pimdb_set_batch(h, S, arr(ctypes.c_int64, self.N), arr(ctypes.c_int32, self.P),
                                       arr(ctypes.c_double, self.beta), arr(ctypes.c_double, self.m),
                                       arr(ctypes.c_double, self.omega_p)), h)
        if threads or per_thread:
            check(self.lib.pimdb_set_tuning(h, int(threads), int(per_thread)), h)
        if split != -1:
            check(self.lib.pimdb_set_split(h, int(split)), h)
        if algorithm != "fast" or shift != "min":
            self._set_algorithm(algorithm, shift)
        self.pair = None
        if pair is not None:
            self.pair = (float(pair[0]), float(pair[1]))
            check(self.lib.pimdb_set_pair_gaussian(h, self.pair[0], self.pair[1]), h)
        self._bind()

    # ------------------------------------------------------------ plumbing
    def _bind(self):
        h = self._h
        if getattr(self, "_captured", False) and getattr(self, "workspace", None) is not None:
            # a captured graph still uses the old workspace: keep it alive
            self._old_workspaces.append(self.workspace)
        nbytes = int(self.lib.pimdb_workspace_bytes(h))
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._stream()
        check(self.lib.pimdb_bind_workspace(h, ctypes.c_void_p(aligned), nbytes), h)
        self.offsets = [int(self.lib.pimdb_system_offset(h, s)) for s in range(self.S)]
        self.total = int(self.lib.pimdb_total_elements(h))

    def set_tuning(self, threads: int, per_thread: int):
        """Change the launch shape.  Graphs captured earlier stay valid: the
        library keeps their tables and this object their workspace."""
        check(self.lib.pimdb_set_tuning(self._h, int(threads), int(per_thread)), self._h)
        self._bind()

    _ALG = {"fast": _lib.PIMDB_ALG_FAST, "original": _lib.PIMDB_ALG_ORIGINAL}
    _SHIFT = {"min": _lib.PIMDB_SHIFT_MIN, "two_term": _lib.PIMDB_SHIFT_TWO_TERM}

    def _set_algorithm(self, algorithm, shift):
        if algorithm not in self._ALG or shift not in self._SHIFT:
            raise ValueError("algorithm must be 'fast' or 'original', shift 'min' or 'two_term'")
        check(self.lib.pimdb_set_algorithm(self._h, self._ALG[algorithm], self._SHIFT[shift]), self._h)

    def set_algorithm(self, algorithm: str, shift: str = "min"):
        """'fast' (the quadratic algorithm, default) or 'original' (the cubic
        comparison path, O(P N^3) time and O(P N^2) workspace); shift 'min' or
        'two_term' selects the original algorithm's shift of the forward
        recurrence.  Rebinds the workspace."""
        self._set_algorithm(algorithm, shift)
        self._bind()

    def set_pair_gaussian(self, g: float, sigma: float = 1.0):
        """Add the scaled pair interaction (1/P) sum_j sum_{a<b} g exp(-r^2 /
        (2 sigma^2)) to every later evaluation (g = 0 removes it).  Rebinds
        the workspace."""
        check(self.lib.pimdb_set_pair_gaussian(self._h, float(g), float(sigma)), self._h)
        self.pair = (float(g), float(sigma)) if g != 0 else None
        self._bind()

    def pair_forces(self, pos, out=None, energy=None):
        """The pair interaction alone: (forces, energies)."""
        out = self.empty() if out is None else out
        energy = torch.empty(self.S, dtype=torch.float64, device=self.device) if energy is None else energy
        self._stream()
        check(self.lib.pimdb_pair_forces(self._h, self._ptr(pos, self.total, "pos"), self._ptr(out, self.total, "forces"),
                                         self._ptr(energy, self.S, "energy")), self._h)
        return out, energy

    @property
    def algorithm(self):
        a, s = ctypes.c_int(), ctypes.c_int()
        check(self.lib.pimdb_get_algorithm(self._h, ctypes.byref(a), ctypes.byref(s)), self._h)
        inv = {v: k for k, v in self._ALG.items()}, {v: k for k, v in self._SHIFT.items()}
        return inv[0][a.value], inv[1][s.value]

    def set_timing(self, enable: bool = True):
        """Record HIP events around the exchange and finalize launches of
        every later eager evaluation (see last_timing)."""
        check(self.lib.pimdb_set_timing(self._h, 1 if enable else 0), self._h)

    def last_timing(self):
        """(exchange launch ms, finalize launch ms) of the last timed eager
        evaluation, from HIP events on the library's stream."""
        a, b = ctypes.c_float(), ctypes.c_float()
        check(self.lib.pimdb_last_timing(self._h, ctypes.byref(a), ctypes.byref(b)), self._h)
        return a.value, b.value

    def set_split(self, blocks_per_helper: int):
        """Split recursions: -1 automatic, 0 never, g >= 1 at most g blocks of
        64 accumulators per helper workgroup (see include/pimdb.h)."""
        check(self.lib.pimdb_set_split(self._h, int(blocks_per_helper)), self._h)
        self._bind()

    @property
    def split(self):
        """(blocks per helper of the current plan, 0 if unsplit; helper
        workgroups per forces call; 1 if every workgroup of the split launch
        has a CU of its own)."""
        g, n, x = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(self.lib.pimdb_get_split(self._h, ctypes.byref(g), ctypes.byref(n), ctypes.byref(x)), self._h)
        return g.value, n.value, x.value

    @property
    def tuning(self):
        t, p = ctypes.c_int(), ctypes.c_int()
        check(self.lib.pimdb_get_tuning(self._h, ctypes.byref(t), ctypes.byref(p)), self._h)
        return t.value, p.value

    def _stream(self):
        if torch.cuda.is_current_stream_capturing():
            self._captured = True
        st = torch.cuda.current_stream(self.device).cuda_stream
        check(self.lib.pimdb_set_stream(self._h, ctypes.c_void_p(st)), self._h)

    def _ptr(self, t, numel, name):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device:
            raise TypeError("%s must be a float64 tensor on %s" % (name, self.device))
        if not t.is_contiguous() or t.numel() != numel:
            raise ValueError("%s must be contiguous with %d elements" % (name, numel))
        return ctypes.c_void_p(t.data_ptr())

    def close(self):
        if getattr(self, "_h", None) is not None:
            self.lib.pimdb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- layout
    def empty(self):
        return torch.empty(self.total, dtype=torch.float64, device=self.device)

    def pack(self, systems: Sequence) -> torch.Tensor:
        """Pack per-system (N, P, 3) arrays into the device SoA layout."""
        if self.S == 1 and not isinstance(systems, (list, tuple)):
            systems = [systems]
        flat = np.empty(self.total, dtype=np.float64)
        for s, R in enumerate(systems):
            R = np.asarray(R, dtype=np.float64)
            assert R.shape == (self.N[s], self.P[s], 3)
            o = self.offsets[s]
            flat[o:o + R.size] = np.transpose(R, (1, 2, 0)).ravel()
        return torch.from_numpy(flat).to(self.device)

    def view(self, flat: torch.Tensor, s: int) -> torch.Tensor:
        """(P, 3, N) view of system s in a packed tensor."""
        o = self.offsets[s]
        n = 3 * self.P[s] * self.N[s]
        return flat[o:o + n].view(self.P[s], 3, self.N[s])

    def unpack(self, flat: torch.Tensor, s: int) -> np.ndarray:
        """System s of a packed tensor as a host (N, P, 3) array."""
        return self.view(flat, s).permute(2, 0, 1).contiguous().cpu().numpy()

    # --------------------------------------------------------- evaluation
    def energy(self, pos, out=None):
        out = torch.empty(self.S, dtype=torch.float64, device=self.device) if out is None else out
        self._stream()
        check(self.lib.pimdb_exchange_energy(self._h, self._ptr(pos, self.total, "pos"),
                                             self._ptr(out, self.S, "energy")), self._h)
        return out

    def forces(self, pos, out=None, energy=None, want_energy=True):
        out = self.empty() if out is None else out
        if energy is None and want_energy:
            energy = torch.empty(self.S, dtype=torch.float64, device=self.device)
        self._stream()
        e_ptr = self._ptr(energy, self.S, "energy") if energy is not None else None
        check(self.lib.pimdb_exchange_forces(self._h, self._ptr(pos, self.total, "pos"),
                                             self._ptr(out, self.total, "forces"), e_ptr), self._h)
        return out, energy

    def forces_batched(self, pos, offsets, out, energy):
        """Forces and energies of systems packed at caller-chosen element
        offsets: `offsets` is a device int64 tensor of S offsets into `pos`
        and `out` (system s occupies 3 P_s N_s elements from offsets[s])."""
        if offsets.dtype != torch.int64 or offsets.device != self.device or offsets.numel() != self.S:
            raise TypeError("offsets must be an int64 tensor of %d entries on %s" % (self.S, self.device))
        for t, name in ((pos, "pos"), (out, "forces")):
            if t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous():
                raise TypeError("%s must be a contiguous float64 tensor on %s" % (name, self.device))
        self._stream()
        check(self.lib.pimdb_exchange_forces_batched(self._h, ctypes.c_void_p(pos.data_ptr()),
                                                     ctypes.c_void_p(offsets.contiguous().data_ptr()),
                                                     ctypes.c_void_p(out.data_ptr()),
                                                     self._ptr(energy, self.S, "energy")), self._h)
        return out, energy

    def forces_static(self, pos, out=None, energy=None, want_energy=True):
        """As forces(), through the entry point that allocates nothing and
        uses the library's static device scratch instead of the bound
        workspace (batches up to _lib.STATIC_SCRATCH_BYTES of scratch)."""
        out = self.empty() if out is None else out
        if energy is None and want_energy:
            energy = torch.empty(self.S, dtype=torch.float64, device=self.device)
        self._stream()
        e_ptr = self._ptr(energy, self.S, "energy") if energy is not None else None
        check(self.lib.pimdb_exchange_forces_static(self._h, self._ptr(pos, self.total, "pos"),
                                                    self._ptr(out, self.total, "forces"), e_ptr), self._h)
        return out, energy

    def state_bytes(self) -> int:
        return int(self.lib.pimdb_state_bytes(self._h))

    def energy_save(self, pos, state, energy):
        self._stream()
        if state.numel() * state.element_size() < self.state_bytes():
            raise ValueError("state buffer too small")
        check(self.lib.pimdb_exchange_energy_save(self._h, self._ptr(pos, self.total, "pos"),
                                                  self._ptr(energy, self.S, "energy"),
                                                  ctypes.c_void_p(state.data_ptr())), self._h)
        return energy

    def adjoint(self, pos, state, grad_energy, out):
        self._stream()
        check(self.lib.pimdb_exchange_adjoint(self._h, self._ptr(pos, self.total, "pos"),
                                              ctypes.c_void_p(state.data_ptr()),
                                              self._ptr(grad_energy, self.S, "grad_energy"),
                                              self._ptr(out, self.total, "grad_pos")), self._h)
        return out

    def md_step(self, pos, vel, forces, energy, dt):
        self._stream()
        e_ptr = self._ptr(energy, self.S, "energy") if energy is not None else None
        check(self.lib.pimdb_md_step(self._h, self._ptr(pos, self.total, "pos"), self._ptr(vel, self.total, "vel"),
                                     self._ptr(forces, self.total, "forces"), e_ptr, float(dt)), self._h)

    def distinguishable(self, pos, out=None, energy=None):
        out = self.empty() if out is None else out
        energy = torch.empty(self.S, dtype=torch.float64, device=self.device) if energy is None else energy
        self._stream()
        check(self.lib.pimdb_distinguishable_forces(self._h, self._ptr(pos, self.total, "pos"),
                                                    self._ptr(out, self.total, "forces"),
                                                    self._ptr(energy, self.S, "energy")), self._h)
        return out, energy

    def debug(self, pos, s, what):
        """Synchronous export of intermediates of system s (see include/pimdb.h)."""
        N = self.N[s]
        n = {1: N * N, 2: N * N, 3: N + 1, 4: N + 2}[int(what)]
        dst = torch.zeros(n, dtype=torch.float64, device=self.device)
        self._stream()
        check(self.lib.pimdb_debug_get(self._h, self._ptr(pos, self.total, "pos"), int(s), int(what),
                                       ctypes.c_void_p(dst.data_ptr())), self._h)
        if what in (1, 2):
            return dst.view(N, N)
        return dst

    def endpoint_springs(self, pos, s, as_float=False, out=None):
        N = self.N[s]
        M = N * (N + 1) // 2
        dt = torch.float32 if as_float else torch.float64
        out = torch.empty(M, dtype=dt, device=self.device) if out is None else out
        self._stream()
        check(self.lib.pimdb_endpoint_springs(self._h, self._ptr(pos, self.total, "pos"), int(s),
                                              1 if as_float else 0, ctypes.c_void_p(out.data_ptr())), self._h)
        return out

    def status(self) -> int:
        self._stream()
        flags = ctypes.c_int32(0)
        rc = self.lib.pimdb_status(self._h, ctypes.byref(flags))
        if rc not in (_lib.PIMDB_OK, _lib.PIMDB_ENONFINITE):
            check(rc, self._h)
        return flags.value
