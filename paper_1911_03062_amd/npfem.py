"""Python binding of libnpfem (ctypes, argument marshalling only).

Every step of the solver runs in the library's HIP kernels; PyTorch supplies device memory
and the current stream. The library must have been built (``build_lib.build()``); importing
this module on a machine without it raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnpfem.so")
HEADER_PATH = os.path.join(HERE, "..", "include", "npfem.h")

STATUS = {0: "NPFEM_OK", -1: "NPFEM_E_INVALID", -2: "NPFEM_E_MESH", -3: "NPFEM_E_NOT_SPD",
          -4: "NPFEM_E_DT", -5: "NPFEM_E_NOMEM", -6: "NPFEM_E_HIP", -7: "NPFEM_E_NONFINITE",
          -8: "NPFEM_E_UNSUPPORTED"}
FORMS = {"plain": 0, "fused": 1}
SOLVES = {"dense": 0, "banded": 1, "auto": 2, "gemv": 3}


class NpfemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class _Mesh(ctypes.Structure):
    _fields_ = [("n_vertices", c_int32), ("n_triangles", c_int32),
                ("rest_xyz", POINTER(c_double)), ("tri", POINTER(c_int32))]


class _Material(ctypes.Structure):
    _fields_ = [("density", c_double), ("shear_B", c_double), ("area_C", c_double),
                ("skalak_D", c_double), ("k_bend", c_double), ("k_vol", c_double),
                ("strain_min", c_double), ("strain_max", c_double), ("pbd_kappa", c_double),
                ("v_max", c_double), ("rayleigh_alpha", c_double), ("rayleigh_beta", c_double),
                ("membrane", c_int32)]

MEMBRANES = {"pd": 0, "skalak": 1}


class _Info(ctypes.Structure):
    _fields_ = [("n_vertices", c_int32), ("n_triangles", c_int32), ("n_hinges", c_int32),
                ("bandwidth", c_int32), ("rest_volume", c_double), ("rest_area", c_double),
                ("vertex_mass", c_double), ("dt", c_double), ("tri_rounds", c_int32),
                ("hinge_rounds", c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libnpfem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1911_03062_amd.build_lib")
    # PyTorch ships its own HIP runtime whose SONAME equals the system one; loading torch
    # first makes the library bind to that same runtime instead of a second copy.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    L.npfem_create_celltype.argtypes = [POINTER(_Mesh), POINTER(_Material), c_double, POINTER(c_void_p)]
    L.npfem_create_celltype.restype = c_int32
    L.npfem_celltype_destroy.argtypes = [c_void_p]
    L.npfem_celltype_destroy.restype = None
    L.npfem_celltype_get_info.argtypes = [c_void_p, POINTER(_Info)]
    L.npfem_celltype_get_info.restype = c_int32
    L.npfem_celltype_get_matrix.argtypes = [c_void_p, POINTER(c_double)]
    L.npfem_celltype_get_matrix.restype = c_int32
    L.npfem_batch_create.argtypes = [c_int32, POINTER(c_void_p), c_int32, c_int32,
                                     POINTER(c_void_p), POINTER(c_int64)]
    L.npfem_batch_create.restype = c_int32
    L.npfem_batch_destroy.argtypes = [c_void_p]
    L.npfem_batch_destroy.restype = None
    L.npfem_batch_vertex_count.argtypes = [c_void_p]
    L.npfem_batch_vertex_count.restype = c_int64
    L.npfem_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32,
                             c_void_p, c_void_p]
    L.npfem_step.restype = c_int32
    L.npfem_step_contacts.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32,
                                      c_void_p, c_void_p, c_void_p, c_void_p]
    L.npfem_step_contacts.restype = c_int32
    L.npfem_batch_set_active.argtypes = [c_void_p, POINTER(c_int32), c_int32, c_void_p]
    L.npfem_batch_set_active.restype = c_int32
    L.npfem_batch_check.argtypes = [c_void_p, c_void_p]
    L.npfem_filter_forces.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
    L.npfem_filter_forces.restype = c_int32
    L.npfem_detect_contacts.argtypes = [c_void_p, c_void_p, c_double, c_double, c_double,
                                        c_void_p, c_void_p, c_void_p]
    L.npfem_detect_contacts.restype = c_int32
    L.npfem_detect_contacts_noalloc.argtypes = [c_void_p, c_void_p, c_double, c_double, c_double,
                                                c_void_p, c_void_p, c_void_p]
    L.npfem_detect_contacts_noalloc.restype = c_int32
    L.npfem_global_solve.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]
    L.npfem_global_solve.restype = c_int32
    L.npfem_batch_get_global_solve.argtypes = [c_void_p, POINTER(c_int32)]
    L.npfem_batch_get_global_solve.restype = c_int32
    L.npfem_batch_check.restype = c_int32
    L.npfem_celltype_cells_per_wave.argtypes = [c_void_p, POINTER(c_int32), c_int32]
    L.npfem_celltype_cells_per_wave.restype = c_int32
    L.npfem_batch_get_cells_per_wave.argtypes = [c_void_p, c_void_p, POINTER(c_int32)]
    L.npfem_batch_get_cells_per_wave.restype = c_int32
    L.npfem_batch_set_cells_per_wave.argtypes = [c_void_p, c_void_p, c_int32]
    L.npfem_batch_set_cells_per_wave.restype = c_int32
    L.npfem_batch_autotune.argtypes = [c_void_p, c_int32, c_int32, c_void_p]
    L.npfem_batch_autotune.restype = c_int32
    L.npfem_graph_create.argtypes = [c_void_p, c_void_p, c_void_p, POINTER(c_void_p), c_int32,
                                     c_double, c_int32, c_void_p, POINTER(c_void_p)]
    L.npfem_graph_create.restype = c_int32
    L.npfem_graph_launch.argtypes = [c_void_p, c_void_p]
    L.npfem_graph_launch.restype = c_int32
    L.npfem_graph_destroy.argtypes = [c_void_p]
    L.npfem_graph_destroy.restype = None
    L.npfem_last_error.argtypes = []
    L.npfem_last_error.restype = c_char_p
    _lib = L
    return L


def header_symbols() -> list[str]:
    """Function names declared in include/npfem.h."""
    src = open(HEADER_PATH).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(npfem_[a-z_0-9]+)\s*\(", src)))


def _check(status: int):
    if status != 0:
        msg = lib().npfem_last_error().decode(errors="replace")
        raise NpfemError(status, msg)


class CellType:
    """A cell type built on the host (mesh validation, rest frames, L and its factors)."""

    def __init__(self, rest_xyz, tri, material, dt: float):
        x = np.ascontiguousarray(rest_xyz, dtype=np.float64)
        t = np.ascontiguousarray(tri, dtype=np.int32)
        if x.ndim != 2 or x.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3:
            raise ValueError("rest_xyz must be [n][3] and tri [m][3]")
        mesh = _Mesh(x.shape[0], t.shape[0], x.ctypes.data_as(POINTER(c_double)),
                     t.ctypes.data_as(POINTER(c_int32)))
        mat = _Material(material.density, material.shear_B, material.area_C, material.skalak_D,
                        material.k_bend, material.k_vol, material.strain_min, material.strain_max,
                        float(getattr(material, "pbd_kappa", 0.0)),
                        float(getattr(material, "v_max", 0.0)),
                        float(getattr(material, "rayleigh_alpha", 0.0)),
                        float(getattr(material, "rayleigh_beta", 0.0)),
                        MEMBRANES[getattr(material, "membrane", "pd")])
        h = c_void_p()
        _check(lib().npfem_create_celltype(ctypes.byref(mesh), ctypes.byref(mat), float(dt),
                                           ctypes.byref(h)))
        self._h = h
        self.dt = float(dt)

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        i = _Info()
        _check(lib().npfem_celltype_get_info(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in _Info._fields_}

    def cells_per_wave(self) -> list:
        """Feasible fused-form layouts (cells per wave), the default first."""
        buf = (c_int32 * 8)()
        n = lib().npfem_celltype_cells_per_wave(self._h, buf, 8)
        if n < 0:
            _check(n)
        return [int(buf[i]) for i in range(min(n, 8))]

    def matrix(self) -> np.ndarray:
        n = self.info()["n_vertices"]
        L = np.empty((n, n), dtype=np.float64)
        _check(lib().npfem_celltype_get_matrix(self._h, L.ctypes.data_as(POINTER(c_double))))
        return L

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.npfem_celltype_destroy(h)
            self._h = None


class Batch:
    """A batch of cells (one type handle per cell) bound to the current HIP device."""

    def __init__(self, cell_types, precision: int = 32, form: str = "fused"):
        self._types = list(cell_types)      # keep the handles alive
        n = len(self._types)
        arr = (c_void_p * max(n, 1))(*[t.handle.value for t in self._types])
        off = np.zeros(n + 1, dtype=np.int64)
        h = c_void_p()
        _check(lib().npfem_batch_create(n, arr, int(precision), FORMS[form], ctypes.byref(h),
                                        off.ctypes.data_as(POINTER(c_int64))))
        self._h = h
        self.offsets = off
        self.n_cells = n
        self.precision = int(precision)
        self.form = form
        self.dt = self._types[0].dt if n else 0.0

    @property
    def vertex_count(self) -> int:
        return int(self.offsets[-1])

    def step(self, x, v, f, dt: float, n_pd_iters: int, vol_area=None, stream=None,
             contacts=None):
        """Advance in place; x, v, f are device tensors [3][V_total] of the batch's dtype.
        contacts = (p [3][V_total], w [V_total]) adds the collision energies."""
        import torch
        dtype = torch.float64 if self.precision == 64 else torch.float32
        cp = cw = 0
        if contacts is not None:
            p_, w_ = contacts
            if not (w_.is_cuda and w_.dtype == dtype and w_.is_contiguous()
                    and tuple(w_.shape) == (self.vertex_count,)):
                raise ValueError(f"contact weights must be a contiguous device tensor [{self.vertex_count}] of {dtype}")
            cp, cw = p_, w_
        for name, t in (("x", x), ("v", v), ("f", f)) + ((("contact points", cp),) if contacts is not None else ()):
            if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()
                    and tuple(t.shape) == (3, self.vertex_count)):
                raise ValueError(f"{name} must be a contiguous device tensor [3][{self.vertex_count}] of {dtype}")
        va = 0
        if vol_area is not None:
            if not (vol_area.is_cuda and vol_area.dtype == torch.float64 and vol_area.is_contiguous()
                    and tuple(vol_area.shape) == (self.n_cells, 2)):
                raise ValueError("vol_area must be a contiguous float64 device tensor [n_cells][2]")
            va = vol_area.data_ptr()
        s = stream if stream is not None else torch.cuda.current_stream()
        if contacts is None:
            _check(lib().npfem_step(self._h, x.data_ptr(), v.data_ptr(), f.data_ptr(), float(dt),
                                    int(n_pd_iters), c_void_p(s.cuda_stream), c_void_p(va)))
        else:
            _check(lib().npfem_step_contacts(self._h, x.data_ptr(), v.data_ptr(), f.data_ptr(),
                                             float(dt), int(n_pd_iters), c_void_p(s.cuda_stream),
                                             c_void_p(va), c_void_p(cp.data_ptr()),
                                             c_void_p(cw.data_ptr())))

    def filter_forces(self, f_in, f_out=None, stream=None):
        """One-ring median filter of external forces [3][V_total] into f_out (default: in
        place); returns f_out."""
        import torch
        dtype = torch.float64 if self.precision == 64 else torch.float32
        f_out = f_in if f_out is None else f_out
        for name, t in (("f_in", f_in), ("f_out", f_out)):
            if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()
                    and tuple(t.shape) == (3, self.vertex_count)):
                raise ValueError(f"{name} must be a contiguous device tensor [3][{self.vertex_count}] of {dtype}")
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().npfem_filter_forces(self._h, f_in.data_ptr(), f_out.data_ptr(),
                                         c_void_p(s.cuda_stream)))
        return f_out

    def detect_contacts(self, x, radius: float, separation: float, weight: float,
                        contact_p=None, contact_w=None, stream=None):
        """Particle-in-kernel contacts from positions x [3][V_total]: returns (contact_p
        [3][V_total], contact_w [V_total]) for step(..., contacts=...), allocated when not
        given."""
        import torch
        dtype = torch.float64 if self.precision == 64 else torch.float32
        if contact_p is None:
            contact_p = torch.empty_like(x)
        if contact_w is None:
            contact_w = torch.empty((self.vertex_count,), dtype=dtype, device=x.device)
        for name, t, shape in (("x", x, (3, self.vertex_count)),
                               ("contact_p", contact_p, (3, self.vertex_count)),
                               ("contact_w", contact_w, (self.vertex_count,))):
            if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and tuple(t.shape) == shape):
                raise ValueError(f"{name} must be a contiguous device tensor {list(shape)} of {dtype}")
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().npfem_detect_contacts(self._h, x.data_ptr(), float(radius), float(separation),
                                           float(weight), contact_p.data_ptr(),
                                           contact_w.data_ptr(), c_void_p(s.cuda_stream)))
        return contact_p, contact_w

    def global_solve(self, rhs, out=None, solve: str = "dense", stream=None):
        """out = L^-1 rhs for every cell's 3 coordinate columns ([3][V_total] device tensors in
        the batch precision), with the dense L^-1 on the matrix cores ("dense", fused batches),
        the dense L^-1 on the vector ALU ("gemv") or the banded Cholesky substitution
        ("banded"); "auto" takes the variant the autotuner timed fastest."""
        import torch
        dtype = torch.float64 if self.precision == 64 else torch.float32
        if out is None:
            out = torch.empty_like(rhs)
        for name, t in (("rhs", rhs), ("out", out)):
            if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()
                    and tuple(t.shape) == (3, self.vertex_count)):
                raise ValueError(f"{name} must be a contiguous device tensor [3][{self.vertex_count}] of {dtype}")
        if solve not in SOLVES:
            raise ValueError(f"solve must be one of {sorted(SOLVES)}")
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().npfem_global_solve(self._h, SOLVES[solve], rhs.data_ptr(), out.data_ptr(),
                                        c_void_p(s.cuda_stream)))
        return out

    def global_solve_choice(self) -> str:
        """The variant global_solve(solve="auto") takes ("dense", "banded" or "gemv")."""
        out = c_int32(0)
        _check(lib().npfem_batch_get_global_solve(self._h, ctypes.byref(out)))
        return {v: k for k, v in SOLVES.items()}[out.value]

    def detect_contacts_noalloc(self, x, radius: float, separation: float, weight: float,
                                contact_p, contact_w, stream=None):
        """detect_contacts on the library's static per-GPU workspace (no device allocation;
        batches of at most 2^19 vertices; overlapping calls on one GPU race). The caller
        provides contact_p [3][V_total] and contact_w [V_total]."""
        import torch
        dtype = torch.float64 if self.precision == 64 else torch.float32
        for name, t, shape in (("x", x, (3, self.vertex_count)),
                               ("contact_p", contact_p, (3, self.vertex_count)),
                               ("contact_w", contact_w, (self.vertex_count,))):
            if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and tuple(t.shape) == shape):
                raise ValueError(f"{name} must be a contiguous device tensor {list(shape)} of {dtype}")
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().npfem_detect_contacts_noalloc(self._h, x.data_ptr(), float(radius),
                                                   float(separation), float(weight),
                                                   contact_p.data_ptr(), contact_w.data_ptr(),
                                                   c_void_p(s.cuda_stream)))
        return contact_p, contact_w

    def _check_state(self, x, v, forces, vol_area):
        import torch
        dtype = torch.float64 if self.precision == 64 else torch.float32
        named = [("x", x), ("v", v)] + [(f"forces[{i}]", t) for i, t in enumerate(forces)]
        for name, t in named:
            if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()
                    and tuple(t.shape) == (3, self.vertex_count)):
                raise ValueError(f"{name} must be a contiguous device tensor [3][{self.vertex_count}] of {dtype}")
        if vol_area is not None and not (vol_area.is_cuda and vol_area.dtype == torch.float64
                                         and vol_area.is_contiguous()
                                         and tuple(vol_area.shape) == (self.n_cells, 2)):
            raise ValueError("vol_area must be a contiguous float64 device tensor [n_cells][2]")

    def cells_per_wave(self, cell_type: CellType) -> int:
        out = c_int32()
        _check(lib().npfem_batch_get_cells_per_wave(self._h, cell_type.handle, ctypes.byref(out)))
        return int(out.value)

    def set_cells_per_wave(self, cell_type: CellType, cells_per_wave: int):
        _check(lib().npfem_batch_set_cells_per_wave(self._h, cell_type.handle, int(cells_per_wave)))

    def autotune(self, n_pd_iters: int, reps: int = 3, stream=None) -> dict:
        """Time every layout of every type and keep the fastest; returns {type handle: gw}."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().npfem_batch_autotune(self._h, int(n_pd_iters), int(reps), c_void_p(s.cuda_stream)))
        seen = []
        for t in self._types:
            if all(t is not u for u in seen):
                seen.append(t)
        return {t.handle.value: self.cells_per_wave(t) for t in seen}

    def graph(self, x, v, forces, dt: float, n_pd_iters: int, vol_area=None) -> "Graph":
        """Record len(forces) steps on these buffers into a HIP graph (see Graph)."""
        return Graph(self, x, v, forces, dt, n_pd_iters, vol_area)

    def set_active(self, cell_ids, stream=None):
        """Step only these cells from now on (None: all cells)."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        if cell_ids is None:
            _check(lib().npfem_batch_set_active(self._h, None, -1, c_void_p(s.cuda_stream)))
            return
        ids = np.ascontiguousarray(cell_ids, dtype=np.int32)
        self._active_ids = ids
        _check(lib().npfem_batch_set_active(self._h, ids.ctypes.data_as(POINTER(c_int32)),
                                            int(ids.size), c_void_p(s.cuda_stream)))

    def check(self, stream=None):
        """Synchronise and raise NpfemError(NPFEM_E_NONFINITE) if a step produced NaN/Inf."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().npfem_batch_check(self._h, c_void_p(s.cuda_stream)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.npfem_batch_destroy(h)
            self._h = None


class Graph:
    """A recorded sequence of steps of one batch on fixed buffers (npfem_graph_create).

    Step s of a replay uses forces[s]; x, v, the force tensors and vol_area are kept alive by
    the graph, and their contents at replay time are what the steps read.
    """

    def __init__(self, batch: Batch, x, v, forces, dt: float, n_pd_iters: int, vol_area=None):
        forces = list(forces)
        batch._check_state(x, v, forces, vol_area)
        arr = (c_void_p * max(len(forces), 1))(*[f.data_ptr() for f in forces])
        h = c_void_p()
        va = vol_area.data_ptr() if vol_area is not None else None
        _check(lib().npfem_graph_create(batch._h, x.data_ptr(), v.data_ptr(), arr, len(forces),
                                        float(dt), int(n_pd_iters), va, ctypes.byref(h)))
        self._h = h
        self._keep = (batch, x, v, forces, vol_area)
        self.n_steps = len(forces)

    def launch(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().npfem_graph_launch(self._h, c_void_p(s.cuda_stream)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.npfem_graph_destroy(h)
            self._h = None


def make_cell_types(type_inputs: dict, dt: float) -> dict:
    """{type_id: CellType} from {type_id: (rest_xyz, tri, material)}."""
    return {k: CellType(x, t, m, dt) for k, (x, t, m) in type_inputs.items()}
