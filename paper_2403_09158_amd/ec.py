"""Python binding of the HIP library (argument marshalling only).

Every step of the solve runs in ``libec.so``; this module converts arguments
(defect record arrays, problem descriptors, stream handles, output buffers)
and raises :class:`EcError` when the library reports an error.  Calling
anything here without the built library raises immediately: there is no
fallback path.  PyTorch, when present, supplies device memory (through the
library's allocator hooks) and streams.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

from .inputs import DEFECT_DTYPE, Problem

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libec.so")

EC_OK, EC_ERR_ARG, EC_ERR_SIZE, EC_ERR_ADMIT, EC_ERR_DEVICE, EC_ERR_STATE = range(6)
STATUS_NAMES = {0: "EC_OK", 1: "EC_ERR_ARG", 2: "EC_ERR_SIZE", 3: "EC_ERR_ADMIT", 4: "EC_ERR_DEVICE", 5: "EC_ERR_STATE"}
NPROF = 8
PROF_FAMILIES = ("raster", "x_forward", "y_pass", "z_pass_green", "x_inverse_stress", "energy_reduce", "self_term", "other")

# Every symbol include/ec.h declares (checked by the CPU test suite).
EXPORTS = (
    "ec_ctx_create",
    "ec_ctx_destroy",
    "ec_ctx_ledger",
    "ec_ctx_graphs",
    "ec_last_error",
    "ec_state_create",
    "ec_state_destroy",
    "ec_state_bytes",
    "ec_solve_fields",
    "ec_interaction_energies",
    "ec_interaction_energies_noalloc",
    "ec_update_defect",
    "ec_update_batch",
    "ec_jump_energies",
    "ec_jump_select",
    "ec_okmc_step",
    "ec_set_dislocations",
    "ec_set_dislocation_paths",
    "ec_dipole_energies",
    "ec_type_store",
    "ec_type_energies",
    "ec_state_footprints",
    "ec_state_field",
    "ec_state_self_terms",
    "ec_profile_enable",
    "ec_profile_select",
    "ec_profile_read",
    "ec_debug_forward",
    "ec_debug_green",
    "ec_debug_inverse",
)


# ec_path of include/ec.h
PATH_DTYPE = np.dtype([("first", np.int32), ("count", np.int32), ("shift", np.float64, 3), ("b", np.float64, 3)])
assert PATH_DTYPE.itemsize == 56


class EcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class CProblem(ctypes.Structure):
    _fields_ = [
        ("n", c_int32),
        ("prec", c_int32),
        ("bc", c_int32),
        ("nyq", c_int32),
        ("L", c_double),
        ("C11", c_double),
        ("C12", c_double),
        ("C44", c_double),
        ("frame", c_double * 9),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p, c_void_p)

_lib = None


def load() -> ctypes.CDLL:
    """Load libec.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2403_09158_amd.build`")
    try:
        # torch bundles its own HIP runtime with the same soname; loading it
        # first makes libec.so bind to that copy instead of a second runtime.
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i64p, i32p = c_void_p, POINTER(c_double), POINTER(c_int64), POINTER(c_int32)
    sig = {
        "ec_ctx_create": (c_int, [c_int, c_size_t, ALLOC_FN, FREE_FN, vp, POINTER(vp)]),
        "ec_ctx_destroy": (None, [vp]),
        "ec_ctx_ledger": (c_int, [vp, POINTER(c_size_t), POINTER(c_size_t)]),
        "ec_ctx_graphs": (c_int, [vp, POINTER(c_int32)]),
        "ec_last_error": (ctypes.c_char_p, []),
        "ec_state_create": (c_int, [vp, POINTER(CProblem), POINTER(vp)]),
        "ec_state_destroy": (None, [vp]),
        "ec_state_bytes": (c_int, [vp, POINTER(c_size_t)]),
        "ec_solve_fields": (c_int, [vp, vp, c_int32, vp, vp, vp, c_int32]),
        "ec_interaction_energies": (c_int, [vp, vp, vp, c_int32]),
        "ec_interaction_energies_noalloc": (c_int, [vp, vp, vp]),
        "ec_update_defect": (c_int, [vp, c_int32, vp, vp, vp, c_int32]),
        "ec_update_batch": (c_int, [vp, vp, vp, c_int32, vp, vp, c_int32]),
        "ec_jump_energies": (c_int, [vp, vp, c_int32, vp, vp, c_int32]),
        "ec_jump_select": (c_int, [vp, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp, c_int32]),
        "ec_okmc_step": (
            c_int,
            [vp, vp, c_int32, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp, vp],
        ),
        "ec_dipole_energies": (c_int, [vp, vp, vp, c_int32]),
        "ec_type_store": (c_int, [vp, vp, vp, i32p]),
        "ec_type_energies": (c_int, [vp, c_int32, vp, c_int32, vp, vp, vp]),
        "ec_set_dislocations": (c_int, [vp, vp, c_int32, vp]),
        "ec_set_dislocation_paths": (c_int, [vp, vp, c_int32, vp, c_int32, vp]),
        "ec_state_footprints": (c_int, [vp, i32p, i32p, c_int64, i64p]),
        "ec_state_field": (c_int, [vp, c_int32, dp]),
        "ec_state_self_terms": (c_int, [vp, dp]),
        "ec_profile_enable": (c_int, [vp, c_int32]),
        "ec_profile_select": (c_int, [vp, c_int32]),
        "ec_profile_read": (c_int, [vp, i64p, dp, dp]),
        "ec_debug_forward": (c_int, [vp, dp, dp]),
        "ec_debug_green": (c_int, [vp, dp, dp]),
        "ec_debug_inverse": (c_int, [vp, dp, dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int):
    if status != EC_OK:
        raise EcError(status, load().ec_last_error().decode(errors="replace"))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def _stream_handle(stream):
    if stream is None:
        try:
            import torch

            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except ImportError:
            pass
        return 0
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _torch_hooks():
    import torch

    # bound now: at interpreter exit the torch module's attributes may be gone
    # before the last library buffers are freed
    _alloc, _delete = torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete

    def alloc(nbytes, stream, user):
        try:
            return _alloc(int(nbytes))
        except Exception:  # reported to the library as an allocation failure
            return None

    def free(ptr, stream, user):
        try:
            _delete(ptr)
        except Exception:
            pass

    return ALLOC_FN(alloc), FREE_FN(free)


def _user_hooks(alloc, free):
    """ctypes hooks around Python callables alloc(nbytes) -> int or None and
    free(ptr)."""

    def a(nbytes, stream, user):
        try:
            return alloc(int(nbytes))
        except Exception:
            return None

    def f(ptr, stream, user):
        free(ptr)

    return ALLOC_FN(a), FREE_FN(f)


class Context:
    """One device: allocator hooks, HBM admission ledger, cached Green windows."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, allocator: str = "torch", hooks=None):
        """allocator: "torch" (its caching allocator), or "hip" (the
        library's own hipMalloc); hooks: a pair of Python callables
        (alloc(nbytes) -> device pointer or None, free(ptr)) used instead."""
        L = load()
        self._hooks = None
        af, ff = ALLOC_FN(), FREE_FN()
        if hooks is not None:
            self._hooks = _user_hooks(*hooks)
            af, ff = self._hooks
        elif allocator == "torch":
            import torch

            if not torch.cuda.is_available():
                raise RuntimeError("no HIP device visible to torch")
            self._hooks = _torch_hooks()
            af, ff = self._hooks
        h = c_void_p()
        _check(L.ec_ctx_create(device, budget_bytes, af, ff, None, ctypes.byref(h)))
        self.h = h

    def ledger(self):
        used, budget = c_size_t(), c_size_t()
        _check(load().ec_ctx_ledger(self.h, ctypes.byref(used), ctypes.byref(budget)))
        return used.value, budget.value

    def graphs(self) -> int:
        """Executable HIP graphs held for batched hops."""
        k = c_int32()
        _check(load().ec_ctx_graphs(self.h, ctypes.byref(k)))
        return k.value

    def close(self):
        if getattr(self, "h", None):
            load().ec_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def as_defects(defects) -> np.ndarray:
    d = np.ascontiguousarray(defects, dtype=DEFECT_DTYPE)
    if d.ndim == 0:
        d = d.reshape(1)
    return d


def update_batch(states, idx, moved, stream=None, outs=None, use_graph=True):
    """Whole-voxel hops of several states of one shape in one batch
    (``ec_update_batch``): ``states`` (k), ``idx`` (k defect indices),
    ``moved`` (k defect records after their hops), ``outs`` (None or k device
    tensors / None for each state's energies).  Nothing is synchronised."""
    k = len(states)
    hs = (c_void_p * k)(*[st.h.value for st in states])
    ix = np.ascontiguousarray(idx, dtype=np.int32)
    mv = as_defects(moved)
    if ix.shape != (k,) or len(mv) != k:
        raise ValueError("states, idx and moved must have the same length")
    eo = None
    if outs is not None:
        eo = (c_void_p * k)(*[None if o is None else o.data_ptr() for o in outs])
    _check(load().ec_update_batch(hs, ix.ctypes.data, mv.ctypes.data, k, _stream_handle(stream), eo,
                                  1 if use_graph else 0))


class State:
    """One replica: resident fields, footprints and energies of a problem."""

    def __init__(self, ctx: Context, problem: Problem):
        self.ctx = ctx
        self.problem = problem
        fr = tuple(getattr(problem, "frame", ()) or ())
        if fr and len(fr) != 9:
            raise ValueError("frame must hold 9 numbers")
        p = CProblem(
            problem.n, problem.prec, problem.bc, problem.nyq, problem.L, problem.C11, problem.C12, problem.C44,
            (c_double * 9)(*(fr or (0.0,) * 9)),
        )
        h = c_void_p()
        _check(load().ec_state_create(ctx.h, ctypes.byref(p), ctypes.byref(h)))
        self.h = h
        self.ndef = 0
        self._jn = 0  # jumps per defect of the last jump_energies call

    @property
    def n(self):
        return self.problem.n

    def close(self):
        if getattr(self, "h", None):
            load().ec_state_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nbytes(self) -> int:
        b = c_size_t()
        _check(load().ec_state_bytes(self.h, ctypes.byref(b)))
        return b.value

    def solve(self, defects, stream=None, eps_out=None, sig_out=None):
        """Full solve.  eps_out / sig_out: None, a torch tensor on the device, or a
        numpy array on the host ([6, n, n, n], float32 for FP32 states, else float64)."""
        d = as_defects(defects)
        on_dev, eps_p, sig_p = 0, None, None
        for out in (eps_out, sig_out):
            if out is not None and not isinstance(out, np.ndarray):
                on_dev = 1
        if eps_out is not None:
            eps_p = eps_out.data_ptr() if on_dev else eps_out.ctypes.data
        if sig_out is not None:
            sig_p = sig_out.data_ptr() if on_dev else sig_out.ctypes.data
        _check(load().ec_solve_fields(self.h, d.ctypes.data, len(d), _stream_handle(stream), eps_p, sig_p, on_dev))
        self.ndef = len(d)

    def energies(self, stream=None, out=None) -> np.ndarray:
        """Interaction energies (eV) of the current defects; host array unless a
        device tensor is passed as ``out``."""
        if out is not None and not isinstance(out, np.ndarray):
            _check(load().ec_interaction_energies(self.h, _stream_handle(stream), out.data_ptr(), 1))
            return out
        E = np.zeros(self.ndef) if out is None else out
        _check(load().ec_interaction_energies(self.h, _stream_handle(stream), E.ctypes.data, 0))
        return E

    def energies_noalloc(self, out, stream=None):
        """Interaction energies written to the device tensor ``out`` (ndef
        float64) by the entry point that allocates nothing; no synchronisation."""
        _check(load().ec_interaction_energies_noalloc(self.h, _stream_handle(stream), out.data_ptr()))
        return out

    def update(self, idx: int, defect, stream=None, energies: bool = True, out=None):
        """Move defect ``idx`` to ``defect``.  Energies of all defects after the
        move: a host array (``energies``), written to a device tensor ``out``
        without synchronising, or not computed."""
        d = as_defects(defect)
        h = _stream_handle(stream)
        if out is not None and not isinstance(out, np.ndarray):
            _check(load().ec_update_defect(self.h, idx, d.ctypes.data, h, out.data_ptr(), 1))
            return out
        if energies or out is not None:
            E = np.zeros(self.ndef) if out is None else out
            _check(load().ec_update_defect(self.h, idx, d.ctypes.data, h, E.ctypes.data, 0))
            return E
        _check(load().ec_update_defect(self.h, idx, d.ctypes.data, h, None, 0))
        return None

    def type_store(self, proto, stream=None) -> int:
        """Store the spectra of the defect type of the one-record array
        ``proto`` at its own centre; returns the type's index."""
        d = as_defects(proto)
        if len(d) != 1:
            raise ValueError("a prototype is one defect record")
        t = c_int32(-1)
        _check(load().ec_type_store(self.h, d.ctypes.data, _stream_handle(stream), ctypes.byref(t)))
        return t.value

    def type_energies(self, type_id: int, X, X_excl=None, stream=None) -> np.ndarray:
        """Energies (eV) of the stored type translated to the positions ``X``
        (k, 3) (nm), with the resident stress (minus the type's own stress at
        ``X_excl`` if given)."""
        x = np.ascontiguousarray(np.atleast_2d(X), dtype=np.float64)
        if x.shape[1] != 3:
            raise ValueError(f"positions must have shape (k, 3), got {x.shape}")
        xe = None if X_excl is None else np.ascontiguousarray(X_excl, dtype=np.float64).reshape(3)
        E = np.zeros(len(x))
        _check(
            load().ec_type_energies(
                self.h, type_id, x.ctypes.data, len(x), None if xe is None else xe.ctypes.data,
                _stream_handle(stream), E.ctypes.data,
            )
        )
        return E

    def jump_energies(self, jumps, stream=None, out=None) -> np.ndarray:
        """Energy change (eV) of every defect for each of its candidate
        whole-voxel jumps, ``jumps`` of shape (ndef, njump, 3) (integer voxel
        offsets); a host array (ndef, njump), or written to a device tensor
        ``out`` without synchronising."""
        j = np.ascontiguousarray(jumps, dtype=np.int32)
        if j.ndim != 3 or j.shape[0] != self.ndef or j.shape[2] != 3:
            raise ValueError(f"jumps must have shape (ndef={self.ndef}, njump, 3), got {j.shape}")
        nj = j.shape[1]
        h = _stream_handle(stream)
        if out is not None and not isinstance(out, np.ndarray):
            _check(load().ec_jump_energies(self.h, j.ctypes.data, nj, h, out.data_ptr(), 1))
            self._jn = nj
            return out
        dE = np.zeros((self.ndef, nj)) if out is None else out
        _check(load().ec_jump_energies(self.h, j.ctypes.data, nj, h, dE.ctypes.data, 0))
        self._jn = nj
        return dE

    def jump_select(self, Em, nu0: float, kT: float, xi=None, stream=None):
        """Biased frequencies (ndef, njump) of the last jump energies and, given
        random numbers ``xi`` in (0, 1] (one per defect), the chosen jump per
        defect (int32 array; None without ``xi``)."""
        nd = self.ndef
        Em = np.ascontiguousarray(np.broadcast_to(np.asarray(Em, dtype=np.float64), (nd,)))
        x = None if xi is None else np.ascontiguousarray(xi, dtype=np.float64)
        if x is not None and x.shape != (nd,):
            raise ValueError(f"xi must have shape ({nd},)")
        nj = self._jn
        nu = np.zeros((nd, nj))
        choice = np.zeros(nd, dtype=np.int32) if x is not None else None
        _check(
            load().ec_jump_select(
                self.h, Em.ctypes.data, float(nu0), float(kT), None if x is None else x.ctypes.data,
                _stream_handle(stream), nu.ctypes.data, None if choice is None else choice.ctypes.data, 0,
            )
        )
        return nu, choice

    def okmc_step(self, jumps, Em, nu0: float, kT: float, u, xi, dt: float = 0.0, stream=None, energies=False):
        """One OkMC time step: Poisson gate with ``u``, frequency-line choice
        with ``xi`` (both (ndef,) in (0, 1]) among ``jumps`` (ndef, njump, 3),
        the chosen jumps made and the field solved again; ``dt`` <= 0 takes
        1 / max nominal frequency.  Returns the jump index per defect (-1: none)
        and, with ``energies``, the energies after the step."""
        nd = self.ndef
        j = np.ascontiguousarray(jumps, dtype=np.int32)
        if j.ndim != 3 or j.shape[0] != nd or j.shape[2] != 3:
            raise ValueError(f"jumps must have shape (ndef={nd}, njump, 3), got {j.shape}")
        Em = np.ascontiguousarray(np.broadcast_to(np.asarray(Em, dtype=np.float64), (nd,)))
        u = np.ascontiguousarray(u, dtype=np.float64)
        x = np.ascontiguousarray(xi, dtype=np.float64)
        if u.shape != (nd,) or x.shape != (nd,):
            raise ValueError(f"u and xi must have shape ({nd},)")
        choice = np.zeros(nd, dtype=np.int32)
        E = np.zeros(nd) if energies else None
        _check(
            load().ec_okmc_step(
                self.h, j.ctypes.data, j.shape[1], Em.ctypes.data, float(nu0), float(kT), float(dt), u.ctypes.data,
                x.ctypes.data, _stream_handle(stream), choice.ctypes.data, None if E is None else E.ctypes.data,
            )
        )
        self._jn = j.shape[1]
        return (choice, E) if energies else choice

    def set_dislocations(self, lines, stream=None):
        """Straight dislocation lines (records of ``inputs.LINE_DTYPE``) whose
        stress is added to every solve of this state; an empty array removes them."""
        from .inputs import LINE_DTYPE

        a = np.ascontiguousarray(np.asarray(lines, dtype=LINE_DTYPE).reshape(-1))
        _check(load().ec_set_dislocations(self.h, a.ctypes.data if len(a) else None, len(a), _stream_handle(stream)))

    def set_dislocation_paths(self, paths, stream=None):
        """Dislocation loops and lines in any direction whose stress is added to
        every solve of this state: ``paths`` is a list of (verts (k, 3) nm,
        shift (3,) nm, b (3,) nm), a loop when shift is zero, a line through the
        periodic cell when shift is a lattice vector of it; [] removes them."""
        recs = np.zeros(len(paths), dtype=PATH_DTYPE)
        vs = []
        first = 0
        for k, (verts, shift, b) in enumerate(paths):
            v = np.asarray(verts, dtype=np.float64).reshape(-1, 3)
            recs[k]["first"], recs[k]["count"] = first, len(v)
            recs[k]["shift"], recs[k]["b"] = shift, b
            vs.append(v)
            first += len(v)
        verts = np.ascontiguousarray(np.concatenate(vs) if vs else np.zeros((0, 3)))
        _check(
            load().ec_set_dislocation_paths(
                self.h, recs.ctypes.data if len(recs) else None, len(recs),
                verts.ctypes.data if len(verts) else None, len(verts), _stream_handle(stream),
            )
        )

    def dipole_energies(self, stream=None, out=None) -> np.ndarray:
        """Dipole-tensor interaction energies (eV) of the current defects; host
        array unless a device tensor is passed as ``out``."""
        if out is not None and not isinstance(out, np.ndarray):
            _check(load().ec_dipole_energies(self.h, _stream_handle(stream), out.data_ptr(), 1))
            return out
        E = np.zeros(self.ndef) if out is None else out
        _check(load().ec_dipole_energies(self.h, _stream_handle(stream), E.ctypes.data, 0))
        return E

    def footprints(self):
        """List of ascending voxel-id arrays, one per defect."""
        L = load()
        counts = np.zeros(max(self.ndef, 1), dtype=np.int32)
        total = c_int64()
        _check(L.ec_state_footprints(self.h, counts.ctypes.data_as(POINTER(c_int32)), None, 0, ctypes.byref(total)))
        ids = np.zeros(max(total.value, 1), dtype=np.int32)
        _check(
            L.ec_state_footprints(
                self.h, counts.ctypes.data_as(POINTER(c_int32)), ids.ctypes.data_as(POINTER(c_int32)), len(ids), ctypes.byref(total)
            )
        )
        out, o = [], 0
        for c in counts[: self.ndef]:
            out.append(ids[o : o + c].astype(np.int64))
            o += c
        return out

    def field(self, which: str = "sigma") -> np.ndarray:
        code = {"sigma": 0, "eps": 1, "eps_star": 2}[which]
        n = self.n
        out = np.zeros((6, n, n, n))
        _check(load().ec_state_field(self.h, code, _dptr(out)))
        return out

    def self_terms(self) -> np.ndarray:
        out = np.zeros(max(self.ndef, 1))
        _check(load().ec_state_self_terms(self.h, _dptr(out)))
        return out[: self.ndef]

    def profile(self, on: bool = True, families=None):
        """Kernel timing on or off; ``families``: names from PROF_FAMILIES to
        time (None: all)."""
        mask = (1 << NPROF) - 1 if families is None else sum(1 << PROF_FAMILIES.index(f) for f in families)
        _check(load().ec_profile_select(self.h, mask))
        _check(load().ec_profile_enable(self.h, 1 if on else 0))

    def profile_read(self) -> dict:
        launches = np.zeros(NPROF, dtype=np.int64)
        ms = np.zeros(NPROF)
        by = np.zeros(NPROF)
        _check(load().ec_profile_read(self.h, launches.ctypes.data_as(POINTER(c_int64)), _dptr(ms), _dptr(by)))
        return {
            name: {"launches": int(launches[i]), "ms": float(ms[i]), "bytes_per_launch": float(by[i])}
            for i, name in enumerate(PROF_FAMILIES)
        }

    # -- single passes ---------------------------------------------------------
    def debug_forward(self, field: np.ndarray) -> np.ndarray:
        n = self.n
        f = np.ascontiguousarray(field, dtype=np.float64).reshape(6, n, n, n)
        out = np.zeros((6, n, n, n // 2 + 1), dtype=np.complex128)
        _check(load().ec_debug_forward(self.h, _dptr(f), out.view(np.float64).ctypes.data_as(POINTER(c_double))))
        return out

    def debug_green(self, spec: np.ndarray) -> np.ndarray:
        n = self.n
        s = np.ascontiguousarray(spec, dtype=np.complex128).reshape(6, n, n, n // 2 + 1)
        out = np.zeros_like(s)
        _check(
            load().ec_debug_green(
                self.h, s.view(np.float64).ctypes.data_as(POINTER(c_double)), out.view(np.float64).ctypes.data_as(POINTER(c_double))
            )
        )
        return out

    def debug_inverse(self, spec: np.ndarray) -> np.ndarray:
        n = self.n
        s = np.ascontiguousarray(spec, dtype=np.complex128).reshape(6, n, n, n // 2 + 1)
        out = np.zeros((6, n, n, n))
        _check(load().ec_debug_inverse(self.h, s.view(np.float64).ctypes.data_as(POINTER(c_double)), _dptr(out)))
        return out
