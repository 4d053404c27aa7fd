"""Simulation: a context of the HIP library plus the torch buffers it lives in."""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import Desc, Params, check, load


def lattice(q: int, phase: str = "d3q15"):
    """(c [q,3] int array, w [q] float array) in the library's velocity order
    (q = the loaded library's phase-lattice size or 27)."""
    lib = load(phase=phase)
    c = (C.c_int32 * (3 * q))()
    w = (C.c_double * q)()
    check(lib.pflbm_lattice(q, c, w), None, "pflbm_lattice")
    return np.array(c[:], dtype=np.int64).reshape(q, 3), np.array(w[:])


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


# storage dtype of the populations of each precision form
_STORAGE_DTYPES = {"fp64": torch.float64, "fp32": torch.float32, "fp16s": torch.float16}


def check_buffer(t, device, name: str, *, numel: Optional[int] = None, dtype=None,
                 min_bytes: Optional[int] = None) -> torch.Tensor:
    """Refuse, before any library call, a caller buffer the kernels would
    read or write out of bounds or misread: not a tensor, on another device,
    not contiguous, of another dtype, of another length (numel) or smaller
    than min_bytes.  Raises ValueError; returns t."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.device != torch.device(device):
        raise ValueError(f"{name}: on {t.device}, the simulation is on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} values, expected {numel}")
    if min_bytes is not None and t.numel() * t.element_size() < min_bytes:
        raise ValueError(f"{name}: {t.numel() * t.element_size()} bytes, needs at least {min_bytes}")
    return t


def _params_struct(p) -> Params:
    get = (lambda k: p[k]) if isinstance(p, dict) else (lambda k: getattr(p, k))
    s = Params()
    s.tau_H, s.tau_L = get("tau_H"), get("tau_L")
    s.mobility, s.xi, s.sigma = get("mobility"), get("xi"), get("sigma")
    s.rho_H, s.rho_L = get("rho_H"), get("rho_L")
    for k, v in enumerate(get("g")):
        s.g[k] = v
    s.s_high = get("s_high")
    for k, v in enumerate(get("fp16_scale_log2")):
        s.fp16_scale_log2[k] = v
    s.normal_eps = get("normal_eps")
    s.s_bulk = (p.get("s_bulk", 0.0) if isinstance(p, dict) else getattr(p, "s_bulk", 0.0))
    s.rho_g_ref = (p.get("rho_g_ref", 0.0) if isinstance(p, dict) else getattr(p, "rho_g_ref", 0.0))
    return s


class Simulation:
    """One lattice on one GPU.

    Fields handed in or out are float64 torch tensors on the context's device
    with shapes [nz, ny, nx] (scalars) and [3, nz, ny, nx] (vectors).

    The library enqueues on the stream that was current at creation.  A call
    made while another stream is current is ordered after the work already on
    that stream and before what is queued on it next, and the tensors it
    touches are marked as in use on the library's stream.
    """

    def __init__(self, nx: int, ny: int, nz: int, periodic=(True, False, True),
                 precision: str = "fp32", collision: str = "mrt", solid=None, params=None,
                 device: str = "cuda:0", streaming: str = "ab", forcing: str = "first",
                 phase_lattice: str = "d3q15"):
        self.streaming = streaming
        self.forcing = forcing
        self.phase_lattice = phase_lattice
        self.lib = load(phase=phase_lattice)
        self.q_h = int(self.lib.pflbm_phase_q())
        self.device = torch.device(device)
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.precision = precision
        pbits = int(bool(periodic[0])) | (int(bool(periodic[1])) << 1) | (int(bool(periodic[2])) << 2)
        self.desc = Desc(nx, ny, nz, pbits, _lib.PRECISIONS[precision],
                         _lib.COLLISIONS[collision], int(solid is not None),
                         _lib.STREAMING[streaming], _lib.FORCING[forcing])
        nbytes = self.lib.pflbm_workspace_bytes(C.byref(self.desc))
        if nbytes == 0:
            raise ValueError(f"invalid lattice description {nx}x{ny}x{nz}")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        check(self.lib.pflbm_create(C.byref(self.desc), _ptr(self.workspace), nbytes,
                                    C.c_void_p(self.stream.cuda_stream), C.byref(ctx)),
              None, "pflbm_create")
        self.ctx = ctx
        _lib.register(ctx, self.lib)
        self._adj_ws = None
        if params is not None:
            self.set_params(params)
        if solid is not None:
            m = torch.as_tensor(np.asarray(solid, dtype=np.uint8)).reshape(-1).to(self.device)
            check_buffer(m, self.device, "solid mask", numel=self.N, dtype=torch.uint8)
            self._mask = m
            self._run("pflbm_set_mask", self.lib.pflbm_set_mask, _ptr(m), keep=(m,))

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                _lib.unregister(self.ctx)
                self.lib.pflbm_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # ---- helpers -------------------------------------------------------------
    def _run(self, name, fn, *args, keep=()):
        cur = torch.cuda.current_stream(self.device)
        other = cur != self.stream
        if other:
            self.stream.wait_stream(cur)
        check(fn(self.ctx, *args), self.ctx, name)
        if other:
            cur.wait_stream(self.stream)
            for t in keep:
                if t is not None:
                    t.record_stream(self.stream)

    def _f64(self, a, components: int, name: str) -> torch.Tensor:
        """FP64 copy (or view) of a field on the simulation's device, flattened;
        its length must be components * N (1 for scalars, 3 for vectors)."""
        t = torch.as_tensor(a, dtype=torch.float64).to(self.device).reshape(-1).contiguous()
        return check_buffer(t, self.device, name, numel=components * self.N)

    def _state_buf(self, t, name: str) -> torch.Tensor:
        return check_buffer(t, self.device, name, min_bytes=self.state_bytes())

    # ---- forward -------------------------------------------------------------
    def set_params(self, p) -> None:
        s = _params_struct(p)
        self._run("pflbm_set_params", self.lib.pflbm_set_params, C.byref(s))

    def init_equilibrium(self, phi0, u0=None, pstar0=None) -> None:
        phi = self._f64(phi0, 1, "phi0")
        u = None if u0 is None else self._f64(u0, 3, "u0")
        p = None if pstar0 is None else self._f64(pstar0, 1, "pstar0")
        self._init_keep = (phi, u, p)   # alive until the kernels have read them
        self._run("pflbm_init_equilibrium", self.lib.pflbm_init_equilibrium, _ptr(phi), _ptr(u),
                  _ptr(p), keep=(phi, u, p))

    def set_check_interval(self, every: int) -> None:
        """Check sum(phi), sum(p*) for NaN/Inf every `every` steps (0 = off)."""
        self._run("pflbm_set_check_interval", self.lib.pflbm_set_check_interval, int(every))

    def step(self, n: int = 1) -> None:
        self._run("pflbm_step", self.lib.pflbm_step, int(n))

    @property
    def step_count(self) -> int:
        return int(self.lib.pflbm_step_count(self.ctx))

    def moments(self):
        nz, ny, nx = self.shape
        phi = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        p = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._run("pflbm_read_moments", self.lib.pflbm_read_moments, _ptr(phi), _ptr(u), _ptr(p),
                  keep=(phi, u, p))
        return phi, u, p

    def phi(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        check_buffer(out, self.device, "phi out", numel=self.N, dtype=torch.float64)
        self._run("pflbm_read_phi", self.lib.pflbm_read_phi, _ptr(out), keep=(out,))
        return out

    def populations(self):
        h = torch.empty((self.q_h, self.N), dtype=torch.float64, device=self.device)
        g = torch.empty((27, self.N), dtype=torch.float64, device=self.device)
        self._run("pflbm_read_populations", self.lib.pflbm_read_populations, _ptr(h), _ptr(g),
                  keep=(h, g))
        return h, g

    def pack_faces(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """The populations that stream across the two z faces of the lattice,
        as a z-slab of a larger one would send them (pflbm_pack_faces): a
        (2, rows, ny, nx) tensor in the storage dtype, face 0 (plane 0,
        c_z = -1) then face 1 (plane nz - 1, c_z = +1), h rows then g rows."""
        need = C.c_size_t()
        check(self.lib.pflbm_pack_faces(self.ctx, None, 0, C.byref(need)), self.ctx, "pflbm_pack_faces")
        dt = _STORAGE_DTYPES[self.precision]
        nz, ny, nx = self.shape
        rows = need.value // (2 * ny * nx * torch.empty((), dtype=dt).element_size())
        if out is None:
            out = torch.empty((2, rows, ny, nx), dtype=dt, device=self.device)
        check_buffer(out, self.device, "face pack", dtype=dt, min_bytes=need.value)
        self._run("pflbm_pack_faces", self.lib.pflbm_pack_faces, _ptr(out),
                  C.c_size_t(out.numel() * out.element_size()), C.byref(need), keep=(out,))
        return out

    def reduce(self) -> np.ndarray:
        out = (C.c_double * 5)()
        self._run("pflbm_reduce", self.lib.pflbm_reduce, out)
        return np.array(out[:])

    def state_bytes(self) -> int:
        return int(self.lib.pflbm_state_bytes(self.ctx))

    def save_state(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        self._state_buf(out, "saved-state buffer")
        self._run("pflbm_save_state", self.lib.pflbm_save_state, _ptr(out), keep=(out,))
        return out

    def load_state(self, buf: torch.Tensor, step_count: int) -> None:
        self._state_buf(buf, "saved state")
        self._run("pflbm_load_state", self.lib.pflbm_load_state, _ptr(buf), int(step_count),
                  keep=(buf,))

    def step_states(self, src: torch.Tensor, dst: torch.Tensor, n: int, flags: int = 0) -> None:
        """One step from saved state `src` (level n) into buffer `dst` (level
        n + 1); flags as in pflbm.h (write src's phi, leave dst's phi unformed)."""
        self._state_buf(src, "source state")
        self._state_buf(dst, "destination state")
        self._run("pflbm_step_states", self.lib.pflbm_step_states, _ptr(src), _ptr(dst), int(n),
                  int(flags), keep=(src, dst))

    def profile_step(self, n: int):
        """Steps n times under HIP events; returns milliseconds
        (collide-stream kernels summed, phi-update kernels summed, total)."""
        out = (C.c_double * 3)()
        self._run("pflbm_profile_step", self.lib.pflbm_profile_step, int(n), out)
        return float(out[0]), float(out[1]), float(out[2])

    def sync(self) -> None:
        self._run("pflbm_sync", self.lib.pflbm_sync)

    # ---- reverse mode ----------------------------------------------------------
    def adjoint_attach(self) -> None:
        n = self.lib.pflbm_adjoint_workspace_bytes(C.byref(self.desc))
        if self._adj_ws is None:
            self._adj_ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        self._run("pflbm_adjoint_attach", self.lib.pflbm_adjoint_attach, _ptr(self._adj_ws), n)

    def adjoint_reset(self) -> None:
        self._run("pflbm_adjoint_reset", self.lib.pflbm_adjoint_reset)

    def adjoint_inject_phi(self, dl_dphi: torch.Tensor) -> None:
        t = self._f64(dl_dphi, 1, "dL/dphi")
        self._inj_keep = t
        self._run("pflbm_adjoint_inject_phi", self.lib.pflbm_adjoint_inject_phi, _ptr(t), keep=(t,))

    def adjoint_step(self, state_n: torch.Tensor, n: int) -> None:
        self._state_buf(state_n, "primal state")
        self._run("pflbm_adjoint_step", self.lib.pflbm_adjoint_step, _ptr(state_n), int(n),
                  keep=(state_n,))

    def adjoint_init(self, u0=None) -> torch.Tensor:
        u = None if u0 is None else self._f64(u0, 3, "u0")
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._run("pflbm_adjoint_init", self.lib.pflbm_adjoint_init, _ptr(u), _ptr(out),
                  keep=(u, out))
        return out

    def adjoint_grads(self):
        """(dL/dM, dL/dsigma, dL/dxi) accumulated since attach/reset."""
        out = (C.c_double * 3)()
        self._run("pflbm_adjoint_grads", self.lib.pflbm_adjoint_grads, out)
        return float(out[0]), float(out[1]), float(out[2])


def from_workload(wl, precision="fp32", collision="mrt", device="cuda:0", params=None,
                  streaming="ab", forcing="first", phase_lattice="d3q15") -> Simulation:
    """Simulation for a workloads.Workload, initialised at equilibrium.
    streaming: "ab" (two buffers, fused step) or "aa" (in place);
    forcing: "first" (first-order source) or "guo" (Guo's full source);
    phase_lattice: "d3q15" or "d3q27" (selects the library build)."""
    sim = Simulation(wl.nx, wl.ny, wl.nz, wl.periodic, precision, collision, wl.solid,
                     params if params is not None else wl.params, device, streaming, forcing,
                     phase_lattice)
    sim.init_equilibrium(wl.phi0, wl.u0, wl.pstar0)
    return sim
