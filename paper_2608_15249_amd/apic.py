"""Thin Python binding of libapic (ctypes). Argument marshalling only.

torch provides device memory and the current HIP stream; every step of the
PIC loop runs in the HIP kernels of libapic.so. There is no CPU fallback: if
the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapic.so")

APIC_FP64 = 0
APIC_MIXED = 1
APIC_BORIS = 0
APIC_HIGUERA_CARY = 1
APIC_ELECTROSTATIC = 0
APIC_ELECTROMAGNETIC = 1

_STATUS = {0: "APIC_OK", -1: "APIC_EINVAL", -2: "APIC_EHIP", -3: "APIC_ENOMEM", -4: "APIC_EOVERFLOW",
           -5: "APIC_EDOMAIN", -6: "APIC_EUNSUPPORTED"}


class ApicError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (_STATUS.get(status, "?"), status, msg))
        self.status = status


class GridDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("vdim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("dt", ctypes.c_double),
                ("qm", ctypes.c_double), ("q_macro", ctypes.c_double), ("rho_ion", ctypes.c_double),
                ("bz", ctypes.c_double), ("prec", ctypes.c_int), ("frac_bits", ctypes.c_int),
                ("tile_x", ctypes.c_int), ("tile_y", ctypes.c_int),
                ("nz", ctypes.c_int), ("lz", ctypes.c_double), ("tile_z", ctypes.c_int),
                ("pusher", ctypes.c_int), ("c_light", ctypes.c_double), ("model", ctypes.c_int),
                ("walls_x", ctypes.c_int)]


class ParticlesC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("cell", ctypes.c_void_p), ("ox", ctypes.c_void_p), ("oy", ctypes.c_void_p),
                ("vx", ctypes.c_void_p), ("vy", ctypes.c_void_p), ("vz", ctypes.c_void_p),
                ("bucket_start", ctypes.c_void_p), ("perm", ctypes.c_void_p),
                ("z", ctypes.c_void_p), ("oz", ctypes.c_void_p)]


class ReplicaC(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("n", ctypes.c_int64), ("lx", ctypes.c_double)]


class BatchStateC(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_void_p), ("ox", ctypes.c_void_p), ("vx", ctypes.c_void_p), ("E", ctypes.c_void_p)]


EXPORTS = ["apic_create", "apic_destroy", "apic_workspace_size", "apic_num_buckets", "apic_frac_bits", "apic_tile_size",
           "apic_sort_by_cell", "apic_deposit", "apic_field_solve", "apic_gather_push", "apic_step",
           "apic_sync_status", "apic_last_error", "apic_profile_enable", "apic_profile_read", "apic_profile_phases",
           "apic_profile_every",
           "apic_batch_create", "apic_batch_destroy", "apic_batch_sizes", "apic_batch_offsets",
           "apic_batch_work_items", "apic_batch_init", "apic_batch_step", "apic_batch_sync_status",
           "apic_batch_last_error", "apic_autotune_tiles", "apic_batch_autotune_chunk",
           "apic_import_state", "apic_adjoint_sizes", "apic_adjoint_forward", "apic_step_adjoint",
           "apic_em_init_fields", "apic_em_gather_push", "apic_em_step", "apic_charge_exact", "apic_q_macro",
           "apic_step_static", "apic_step_pair"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libapic.so and declare the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libapic.so is not built (%s); run __graft_entry__.build()" % path)
    L = ctypes.CDLL(path)
    vp, i64, dbl, cint = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    P = ctypes.POINTER
    sigs = {
        "apic_create": ([P(GridDesc), i64, P(vp)], cint),
        "apic_destroy": ([vp], None),
        "apic_workspace_size": ([vp, P(ctypes.c_size_t)], cint),
        "apic_num_buckets": ([vp], i64),
        "apic_frac_bits": ([vp], cint),
        "apic_q_macro": ([vp], dbl),
        "apic_tile_size": ([vp, cint], cint),
        "apic_sort_by_cell": ([vp, P(ParticlesC), vp, vp], cint),
        "apic_deposit": ([vp, P(ParticlesC), vp, vp], cint),
        "apic_field_solve": ([vp, vp, vp, vp, vp, vp, vp], cint),
        "apic_gather_push": ([vp, P(ParticlesC), vp, dbl, cint, vp], cint),
        "apic_step": ([vp, P(ParticlesC), vp, vp, vp, cint, vp, vp, vp], cint),
        "apic_sync_status": ([vp, vp], cint),
        "apic_last_error": ([vp], ctypes.c_char_p),
        "apic_profile_enable": ([vp, cint], cint),
        "apic_profile_read": ([vp, P(ctypes.c_double), P(cint)], cint),
        "apic_profile_every": ([vp, cint], cint),
        "apic_profile_phases": ([vp, cint], cint),
        "apic_batch_create": ([P(ReplicaC), cint, dbl, dbl, dbl, cint, P(vp)], cint),
        "apic_batch_destroy": ([vp], None),
        "apic_batch_sizes": ([vp, P(i64), P(i64), P(ctypes.c_size_t)], cint),
        "apic_batch_offsets": ([vp, P(i64), P(i64)], cint),
        "apic_batch_work_items": ([vp], cint),
        "apic_batch_init": ([vp, P(BatchStateC), vp, vp], cint),
        "apic_batch_step": ([vp, P(BatchStateC), cint, vp, vp, vp, vp, cint], cint),
        "apic_batch_sync_status": ([vp, vp], cint),
        "apic_batch_last_error": ([vp], ctypes.c_char_p),
        "apic_import_state": ([vp, vp, vp, vp, vp, vp, vp, P(ParticlesC), vp], cint),
        "apic_adjoint_sizes": ([vp, cint, cint, P(ctypes.c_size_t), P(ctypes.c_size_t)], cint),
        "apic_adjoint_forward": ([vp, P(ParticlesC), cint, cint, vp, vp, vp, vp, vp], cint),
        "apic_step_adjoint": ([vp, vp, cint, cint, dbl, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp], cint),
        "apic_autotune_tiles": ([P(GridDesc), P(ParticlesC), cint, P(cint), P(cint), P(cint), P(dbl), vp], cint),
        "apic_em_init_fields": ([vp, P(ParticlesC), vp, vp, vp], cint),
        "apic_em_gather_push": ([vp, P(ParticlesC), vp, dbl, cint, vp], cint),
        "apic_em_step": ([vp, P(ParticlesC), vp, vp, cint, vp, vp, vp], cint),
        "apic_charge_exact": ([vp, P(i64), P(i64), vp], cint),
        "apic_step_static": ([vp, P(ParticlesC), vp, vp, vp, cint, vp, vp], cint),
        "apic_step_pair": ([vp, P(ParticlesC), P(ParticlesC), vp, vp, vp, cint, vp, P(cint), vp, vp], cint),
        "apic_batch_autotune_chunk": ([P(ReplicaC), cint, dbl, dbl, dbl, P(BatchStateC), cint, P(cint), P(dbl), vp],
                                      cint),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    if path == LIB_PATH:
        _lib = L
    return L


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _need(t, dtype, numel, name, optional=False):
    """Raise ApicError unless t is a contiguous device tensor of dtype with at
    least numel elements (None passes when optional): the kernels read and
    write exactly that many elements through its pointer."""
    if t is None:
        if optional:
            return
        raise ApicError(-1, "%s is required" % name)
    import torch
    if t.device.type != "cuda":
        raise ApicError(-1, "%s must be a device tensor (got %s)" % (name, t.device))
    if t.dtype != dtype:
        raise ApicError(-1, "%s must be %s (got %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ApicError(-1, "%s must be contiguous" % name)
    if t.numel() < numel:
        raise ApicError(-1, "%s holds %d elements, %d needed" % (name, t.numel(), numel))


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One plasma on the GPU: owns the libapic context and its workspace."""

    def __init__(self, *, dim, vdim, nx, ny, lx, ly, dt, n, qm=-1.0, q_macro=None, rho_ion=1.0, bz=0.0,
                 precision="mixed", frac_bits=0, tile=(0, 0), device="cuda", nz=1, lz=1.0, pusher="boris",
                 c_light=0.0, model="es", walls=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libapic needs a HIP GPU; none is visible")
        self.L = load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.mixed = precision == "mixed"
        if q_macro is None:
            q_macro = 0.0       # the library's neutralising default
        tz = tile[2] if len(tile) > 2 else 0
        self.desc = GridDesc(dim, vdim, nx, ny if dim >= 2 else 1, lx, ly if dim >= 2 else 1.0, dt, qm, q_macro,
                             rho_ion, bz, APIC_MIXED if self.mixed else APIC_FP64, frac_bits, tile[0], tile[1],
                             nz if dim == 3 else 1, lz if dim == 3 else 1.0, tz,
                             APIC_HIGUERA_CARY if pusher == "hc" else APIC_BORIS, float(c_light),
                             APIC_ELECTROMAGNETIC if model == "em" else APIC_ELECTROSTATIC, 1 if walls else 0)
        self.model = model
        self.walls = bool(walls)
        self.pusher, self.c_light = pusher, float(c_light)
        self.n = int(n)
        h = ctypes.c_void_p()
        st = self.L.apic_create(ctypes.byref(self.desc), self.n, ctypes.byref(h))
        if st != 0:
            raise ApicError(st, "apic_create rejected the descriptor")
        self.h = h
        sz = ctypes.c_size_t()
        self._check(self.L.apic_workspace_size(self.h, ctypes.byref(sz)))
        self.ws = torch.empty(max(int(sz.value), 256), dtype=torch.uint8, device=self.device)
        self.nbuckets = int(self.L.apic_num_buckets(self.h))
        self.frac_bits = int(self.L.apic_frac_bits(self.h))
        self.q_macro = float(self.L.apic_q_macro(self.h))
        self.tile = tuple(int(self.L.apic_tile_size(self.h, a)) for a in range(dim))
        self.dim, self.vdim, self.nx = dim, vdim, nx
        self.ny = ny if dim >= 2 else 1
        self.nz = nz if dim == 3 else 1
        # grid arrays of a walls context are the odd extension along x (2 nx nodes per row)
        self.nx_grid = 2 * nx if self.walls else nx
        self.G = self.nx_grid * self.ny * self.nz

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.L.apic_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            msg = self.L.apic_last_error(self.h)
            raise ApicError(st, msg.decode() if msg else "")

    def sync(self):
        self._check(self.L.apic_sync_status(self.h, _stream()))

    def charge_exact(self):
        """Exact charge of the last mixed-path field solve: (whole particles,
        remainder in units of 2^-(S dim) particle), from apic_charge_exact."""
        w, f = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.L.apic_charge_exact(self.h, ctypes.byref(w), ctypes.byref(f), _stream()))
        return int(w.value), int(f.value)

    def profile_enable(self, max_steps: int):
        self._check(self.L.apic_profile_enable(self.h, int(max_steps)))

    def profile_phases(self, all_phases: bool):
        """Events around every phase (True, the default) or only around the
        push pass (False: the cheaper form for throughput runs)."""
        self._check(self.L.apic_profile_phases(self.h, 1 if all_phases else 0))

    def profile_every(self, every: int):
        """Profile one step in every `every` (1: each step)."""
        self._check(self.L.apic_profile_every(self.h, int(every)))

    def profile_read(self):
        """Summed milliseconds per phase (count, scan, push, field) and steps."""
        ms = (ctypes.c_double * 4)()
        nst = ctypes.c_int()
        self._check(self.L.apic_profile_read(self.h, ms, ctypes.byref(nst)))
        return list(ms), int(nst.value)

    # -- entry points -------------------------------------------------------
    def sort_by_cell(self, parts: "Particles", perm=None):
        _need(perm, self.torch.int32, self.n, "perm", optional=True)
        s = parts.struct(perm=perm)
        self._check(self.L.apic_sort_by_cell(self.h, ctypes.byref(s), ctypes.c_void_p(self.ws.data_ptr()), _stream()))

    def deposit(self, parts: "Particles", rho, tiled=True):
        t = self.torch
        _need(rho, t.int64 if self.mixed else t.float64, self.G, "rho")
        s = parts.struct(tiled=tiled)
        self._check(self.L.apic_deposit(self.h, ctypes.byref(s), ctypes.c_void_p(rho.data_ptr()), _stream()))

    def field_solve(self, rho, E, E32=None, we=None):
        t = self.torch
        _need(rho, t.int64 if self.mixed else t.float64, self.G, "rho")
        _need(E, t.float64, self.dim * self.G, "E")
        _need(E32, t.float32, self.dim * self.G, "E32", optional=True)
        _need(we, t.float64, 1, "we", optional=True)
        self._check(self.L.apic_field_solve(self.h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(E.data_ptr()),
                                            ctypes.c_void_p(_ptr(E32)), ctypes.c_void_p(_ptr(we)),
                                            ctypes.c_void_p(self.ws.data_ptr()), _stream()))

    def gather_push(self, parts: "Particles", E, dt_scale=1.0, move=True, tiled=True):
        t = self.torch
        _need(E, t.float32 if self.mixed else t.float64, self.dim * self.G, "E")
        s = parts.struct(tiled=tiled)
        self._check(self.L.apic_gather_push(self.h, ctypes.byref(s), ctypes.c_void_p(E.data_ptr()),
                                            float(dt_scale), 1 if move else 0, _stream()))

    def autotune_tiles(self, parts: "Particles", nsteps: int = 5):
        """Fastest sort-bucket tile for this plasma, timed on a copy of
        `parts` (apic_autotune_tiles). Returns (tile, ms_per_step) with tile
        (tile_x, tile_y) below 3D and (tile_x, tile_y, tile_z) in 3D;
        ms_per_step is -1 when the pick came from the process cache."""
        s = parts.struct()
        tx, ty, tz, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        st = self.L.apic_autotune_tiles(ctypes.byref(self.desc), ctypes.byref(s), int(nsteps), ctypes.byref(tx),
                                        ctypes.byref(ty), ctypes.byref(tz), ctypes.byref(ms), _stream())
        if st != 0:
            raise ApicError(st, "apic_autotune_tiles found no runnable tile")
        tile = (int(tx.value), int(ty.value)) + ((int(tz.value),) if self.dim == 3 else ())
        return tile, float(ms.value)

    def import_state(self, parts: "Particles", x, y, vx, vy=None, vz=None, z=None):
        """Physical FP64 device state -> this context's representation (apic_import_state)."""
        t = self.torch
        for a, name, on in ((x, "x", True), (y, "y", self.dim >= 2), (z, "z", self.dim == 3), (vx, "vx", True),
                            (vy, "vy", self.vdim >= 2), (vz, "vz", self.vdim >= 3)):
            _need(a, t.float64, self.n, name, optional=not on)
        s = parts.struct()
        self._check(self.L.apic_import_state(self.h, ctypes.c_void_p(_ptr(x)), ctypes.c_void_p(_ptr(y)),
                                             ctypes.c_void_p(_ptr(z)),
                                             ctypes.c_void_p(_ptr(vx)), ctypes.c_void_p(_ptr(vy)),
                                             ctypes.c_void_p(_ptr(vz)), ctypes.byref(s), _stream()))

    def adjoint_sizes(self, nsteps: int, stride: int):
        ck, ws = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(self.L.apic_adjoint_sizes(self.h, int(nsteps), int(stride), ctypes.byref(ck), ctypes.byref(ws)))
        return int(ck.value), int(ws.value)

    def adjoint_forward(self, parts: "Particles", nsteps, stride, ckpt, ws, W=None, E_out=None):
        t = self.torch
        ck, wb = self.adjoint_sizes(nsteps, stride)
        _need(ckpt, t.uint8, ck, "ckpt")
        _need(ws, t.uint8, wb, "ws")
        _need(W, t.float64, 1, "W", optional=True)
        _need(E_out, t.float64, self.dim * self.G, "E_out", optional=True)
        s = parts.struct()
        self._check(self.L.apic_adjoint_forward(self.h, ctypes.byref(s), int(nsteps), int(stride),
                                                ctypes.c_void_p(ckpt.data_ptr()), ctypes.c_void_p(_ptr(W)),
                                                ctypes.c_void_p(_ptr(E_out)), ctypes.c_void_p(ws.data_ptr()),
                                                _stream()))

    def step_adjoint(self, ckpt, nsteps, stride, ws, lam_x, lam_y, lam_vx, lam_vy=None, lam_vz=None, seed=1.0,
                     dx_ddelta0=None, dy_ddelta0=None, grad_delta0=None, lam_z=None):
        t = self.torch
        ck, wb = self.adjoint_sizes(nsteps, stride)
        _need(ckpt, t.uint8, ck, "ckpt")
        _need(ws, t.uint8, wb, "ws")
        for a, name, on in ((lam_x, "lam_x", True), (lam_y, "lam_y", self.dim >= 2), (lam_z, "lam_z", self.dim == 3),
                            (lam_vx, "lam_vx", True), (lam_vy, "lam_vy", self.vdim >= 2),
                            (lam_vz, "lam_vz", self.vdim >= 3),
                            (dx_ddelta0, "dx_ddelta0", grad_delta0 is not None),
                            (dy_ddelta0, "dy_ddelta0", grad_delta0 is not None and self.dim >= 2)):
            _need(a, t.float64, self.n, name, optional=not on)
        _need(grad_delta0, t.float64, 1, "grad_delta0", optional=True)
        self._check(self.L.apic_step_adjoint(self.h, ctypes.c_void_p(ckpt.data_ptr()), int(nsteps), int(stride),
                                             float(seed), ctypes.c_void_p(_ptr(lam_x)), ctypes.c_void_p(_ptr(lam_y)),
                                             ctypes.c_void_p(_ptr(lam_z)), ctypes.c_void_p(_ptr(lam_vx)), ctypes.c_void_p(_ptr(lam_vy)),
                                             ctypes.c_void_p(_ptr(lam_vz)), ctypes.c_void_p(_ptr(dx_ddelta0)),
                                             ctypes.c_void_p(_ptr(dy_ddelta0)), ctypes.c_void_p(_ptr(grad_delta0)),
                                             ctypes.c_void_p(ws.data_ptr()), _stream()))

    def em_init_fields(self, parts: "Particles", F):
        _need(F, self.torch.float64, 6 * self.G, "F")
        s = parts.struct(tiled=False)
        self._check(self.L.apic_em_init_fields(self.h, ctypes.byref(s), ctypes.c_void_p(F.data_ptr()),
                                               ctypes.c_void_p(self.ws.data_ptr()), _stream()))

    def em_gather_push(self, parts: "Particles", F, dt_scale=1.0, move=True):
        _need(F, self.torch.float64, 6 * self.G, "F")
        s = parts.struct(tiled=False)
        self._check(self.L.apic_em_gather_push(self.h, ctypes.byref(s), ctypes.c_void_p(F.data_ptr()),
                                               float(dt_scale), 1 if move else 0, _stream()))

    def em_step(self, parts: "Particles", F, nsteps, diag=None, J=None, perm=None):
        t = self.torch
        _need(F, t.float64, 6 * self.G, "F")
        _need(J, t.float64, 3 * self.G, "J", optional=True)
        _need(diag, t.float64, 4 * max(int(nsteps), 0), "diag", optional=True)
        _need(perm, t.int32, self.n, "perm", optional=True)
        s = parts.struct(perm=perm)
        self._check(self.L.apic_em_step(self.h, ctypes.byref(s), ctypes.c_void_p(F.data_ptr()),
                                        ctypes.c_void_p(_ptr(J)), int(nsteps), ctypes.c_void_p(_ptr(diag)),
                                        ctypes.c_void_p(self.ws.data_ptr()), _stream()))

    def _check_step(self, E, E32, nsteps, diag, rho, perm):
        t = self.torch
        _need(E, t.float64, self.dim * self.G, "E")
        _need(E32, t.float32, self.dim * self.G, "E32", optional=True)
        _need(diag, t.float64, 4 * max(int(nsteps), 0), "diag", optional=True)
        _need(rho, t.int64 if self.mixed else t.float64, self.G, "rho", optional=True)
        _need(perm, t.int32, self.n, "perm", optional=True)

    def step(self, parts: "Particles", E, E32, nsteps, diag=None, rho=None, perm=None):
        self._check_step(E, E32, nsteps, diag, rho, perm)
        s = parts.struct(perm=perm)
        self._check(self.L.apic_step(self.h, ctypes.byref(s), ctypes.c_void_p(_ptr(rho)), ctypes.c_void_p(E.data_ptr()),
                                     ctypes.c_void_p(_ptr(E32)), int(nsteps), ctypes.c_void_p(_ptr(diag)),
                                     ctypes.c_void_p(self.ws.data_ptr()), _stream()))


    def step_pair(self, parts: "Particles", other: "Particles", E, E32, nsteps, diag=None, rho=None, perm=None):
        """nsteps cycles alternating between two particle buffers
        (apic_step_pair): returns the buffer that holds the state afterwards
        (``other`` for an odd count), with no copy back."""
        self._check_step(E, E32, nsteps, diag, rho, perm)
        if other is parts:
            raise ApicError(-1, "step_pair needs two distinct particle buffers")
        s = parts.struct(perm=perm)
        q = other.struct()
        in_q = ctypes.c_int(0)
        self._check(self.L.apic_step_pair(self.h, ctypes.byref(s), ctypes.byref(q), ctypes.c_void_p(_ptr(rho)),
                                          ctypes.c_void_p(E.data_ptr()), ctypes.c_void_p(_ptr(E32)), int(nsteps),
                                          ctypes.c_void_p(_ptr(diag)), ctypes.byref(in_q),
                                          ctypes.c_void_p(self.ws.data_ptr()), _stream()))
        return other if in_q.value else parts

    def step_static(self, parts: "Particles", E, E32, nsteps, diag=None, rho=None, perm=None):
        """apic_step on the library's fixed device workspace (apic_step_static:
        no allocation, for callers that cannot allocate)."""
        self._check_step(E, E32, nsteps, diag, rho, perm)
        s = parts.struct(perm=perm)
        self._check(self.L.apic_step_static(self.h, ctypes.byref(s), ctypes.c_void_p(_ptr(rho)),
                                            ctypes.c_void_p(E.data_ptr()), ctypes.c_void_p(_ptr(E32)), int(nsteps),
                                            ctypes.c_void_p(_ptr(diag)), _stream()))


class Batch:
    """Many 1D1V replicas on the GPU (apic_batch_*): packed device state."""

    def __init__(self, reps, dt, qm=-1.0, rho_ion=1.0, chunk=0, device="cuda"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libapic needs a HIP GPU; none is visible")
        self.L = load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.nrep = len(reps)
        self.params = (float(dt), float(qm), float(rho_ion))
        arr = (ReplicaC * self.nrep)(*[ReplicaC(int(nx), int(n), float(lx)) for nx, n, lx in reps])
        self.reps_c = arr
        h = ctypes.c_void_p()
        st = self.L.apic_batch_create(arr, self.nrep, float(dt), float(qm), float(rho_ion), int(chunk),
                                      ctypes.byref(h))
        if st != 0:
            raise ApicError(st, "apic_batch_create rejected the replicas")
        self.h = h
        nt, gt, ws = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        self._check(self.L.apic_batch_sizes(h, ctypes.byref(nt), ctypes.byref(gt), ctypes.byref(ws)))
        self.n_total, self.g_total = int(nt.value), int(gt.value)
        po = (ctypes.c_int64 * (self.nrep + 1))()
        go = (ctypes.c_int64 * (self.nrep + 1))()
        self._check(self.L.apic_batch_offsets(h, po, go))
        self.part_off = np.array(list(po), dtype=np.int64)
        self.grid_off = np.array(list(go), dtype=np.int64)
        dev = self.device
        self.ws = torch.zeros(max(int(ws.value), 256), dtype=torch.uint8, device=dev)
        self.cell = torch.zeros(self.n_total, dtype=torch.int32, device=dev)
        self.ox = torch.zeros(self.n_total, dtype=torch.float32, device=dev)
        self.vx = torch.zeros(self.n_total, dtype=torch.float32, device=dev)
        self.E = torch.zeros(self.g_total, dtype=torch.float64, device=dev)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.L.apic_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            msg = self.L.apic_batch_last_error(self.h)
            raise ApicError(st, msg.decode() if msg else "")

    def _state(self):
        return BatchStateC(self.cell.data_ptr(), self.ox.data_ptr(), self.vx.data_ptr(), self.E.data_ptr())

    def upload(self, cell, ox, vx):
        t = self.torch
        self.cell.copy_(t.from_numpy(np.ascontiguousarray(cell, dtype=np.int32)).to(self.device))
        self.ox.copy_(t.from_numpy(np.ascontiguousarray(ox, dtype=np.float32)).to(self.device))
        self.vx.copy_(t.from_numpy(np.ascontiguousarray(vx, dtype=np.float32)).to(self.device))

    def init(self):
        st = self._state()
        self._check(self.L.apic_batch_init(self.h, ctypes.byref(st), ctypes.c_void_p(self.ws.data_ptr()), _stream()))

    def step(self, nsteps, diag=None, rho=None, use_graph=True):
        st = self._state()
        self._check(self.L.apic_batch_step(self.h, ctypes.byref(st), int(nsteps), ctypes.c_void_p(_ptr(diag)),
                                           ctypes.c_void_p(_ptr(rho)), ctypes.c_void_p(self.ws.data_ptr()),
                                           _stream(), 1 if use_graph else 0))

    def sync(self):
        self._check(self.L.apic_batch_sync_status(self.h, _stream()))

    def work_items(self):
        return int(self.L.apic_batch_work_items(self.h))

    def autotune_chunk(self, nsteps: int = 5):
        """Fastest work-item size for these replicas, timed on a copy of the
        uploaded state (apic_batch_autotune_chunk). Returns (chunk, ms_per_step);
        ms_per_step is -1 when the pick came from the process cache."""
        st = self._state()
        ch, ms = ctypes.c_int(), ctypes.c_double()
        dt, qm, rho_ion = self.params
        r = self.L.apic_batch_autotune_chunk(self.reps_c, self.nrep, dt, qm, rho_ion, ctypes.byref(st), int(nsteps),
                                             ctypes.byref(ch), ctypes.byref(ms), _stream())
        if r != 0:
            raise ApicError(r, "apic_batch_autotune_chunk found no runnable chunk size")
        return int(ch.value), float(ms.value)


class Particles:
    """Device SoA particle arrays for one Context (torch tensors)."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        t = ctx.torch
        n, dev = ctx.n, ctx.device
        r = t.float32 if ctx.mixed else t.float64
        self.x = self.y = self.z = self.cell = self.ox = self.oy = self.oz = None
        if ctx.mixed:
            self.cell = t.zeros(n, dtype=t.int32, device=dev)
            self.ox = t.zeros(n, dtype=t.float32, device=dev)
            if ctx.dim >= 2:
                self.oy = t.zeros(n, dtype=t.float32, device=dev)
            if ctx.dim == 3:
                self.oz = t.zeros(n, dtype=t.float32, device=dev)
        else:
            self.x = t.zeros(n, dtype=t.float64, device=dev)
            if ctx.dim >= 2:
                self.y = t.zeros(n, dtype=t.float64, device=dev)
            if ctx.dim == 3:
                self.z = t.zeros(n, dtype=t.float64, device=dev)
        self.vx = t.zeros(n, dtype=r, device=dev)
        self.vy = t.zeros(n, dtype=r, device=dev) if ctx.vdim >= 2 else None
        self.vz = t.zeros(n, dtype=r, device=dev) if ctx.vdim >= 3 else None
        self.bucket_start = t.zeros(ctx.nbuckets + 1, dtype=t.int32, device=dev)

    def struct(self, perm=None, tiled=True) -> ParticlesC:
        return ParticlesC(self.ctx.n, _ptr(self.x), _ptr(self.y), _ptr(self.cell), _ptr(self.ox), _ptr(self.oy),
                          _ptr(self.vx), _ptr(self.vy), _ptr(self.vz),
                          _ptr(self.bucket_start) if tiled else None, _ptr(perm), _ptr(self.z), _ptr(self.oz))

    def upload(self, x=None, y=None, vx=None, vy=None, vz=None, cell=None, ox=None, oy=None, z=None, oz=None):
        t = self.ctx.torch
        dev = self.ctx.device

        def put(dst, src):
            if src is not None and dst is not None:
                dst.copy_(t.from_numpy(np.ascontiguousarray(src)).to(dev, dst.dtype))

        put(self.x, x)
        put(self.y, y)
        put(self.cell, cell)
        put(self.ox, ox)
        put(self.oy, oy)
        put(self.z, z)
        put(self.oz, oz)
        put(self.vx, vx)
        put(self.vy, vy)
        put(self.vz, vz)

    def download(self):
        g = lambda a: None if a is None else a.cpu().numpy()
        return {k: g(getattr(self, k))
                for k in ("x", "y", "z", "cell", "ox", "oy", "oz", "vx", "vy", "vz", "bucket_start")}
