"""Python binding of libmbks (argument marshalling only).

Every operation runs in the HIP library; this module converts the problem
dictionary into the C description, hands torch device buffers and the current
stream to the C entry points, and turns status codes into exceptions.  It never
computes a step of the method itself; if the library is missing it raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_uint64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbks.so")

MB_FP64, MB_FP32, MB_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": MB_FP64, "fp32": MB_FP32, "bf16x3": MB_BF16X3}
STATUS = {0: "MB_OK", -1: "MB_ERR_INVALID_ARG", -2: "MB_ERR_NOT_SPD", -3: "MB_ERR_NOT_CONVERGED",
          -4: "MB_ERR_NONFINITE", -5: "MB_ERR_OOM", -6: "MB_ERR_HIP", -7: "MB_ERR_NO_DEVICE"}
MB_MAX_GAUSS = 4

# every symbol the C header declares
EXPORTS = ("mb_init", "mb_problem_create", "mb_problem_destroy", "mb_problem_dims", "mb_problem_gvectors",
           "mb_problem_zrule", "mb_problem_zbands", "mb_problem_projectors", "mb_problem_augmentation",
           "mb_problem_set_potential",
           "mb_problem_reserve", "hpsi_apply", "hpsi_apply_gamma", "hpsi_apply_noalloc", "spsi_apply", "s_solve", "mb_lanczos_default_opts", "lanczos_lowest",
           "density_accumulate", "hartree_potential", "mb_tune_get", "mb_tune_set", "mb_tune_save",
           "mb_tune_load", "mb_batch_bind", "hpsi_apply_batched_bound", "mb_batch_create", "mb_batch_destroy", "hpsi_apply_batched", "lanczos_lowest_batched", "mb_autotune",
           "mb_small_geneig", "mb_timer_enable", "mb_timer_read", "mb_last_error", "mb_wire_create",
           "mb_wire_dims")


class MbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class MbSpecies(ctypes.Structure):
    _fields_ = [("ngauss", c_int32), ("gauss_A", c_double * MB_MAX_GAUSS), ("gauss_w", c_double * MB_MAX_GAUSS),
                ("nonlocal_", c_int32), ("alpha_s", c_double), ("alpha_p", c_double), ("E_s", c_double),
                ("E_p", c_double), ("q_s", c_double), ("q_p", c_double)]


class MbAtom(ctypes.Structure):
    _fields_ = [("species", c_int32), ("pos", c_double * 3)]


class MbDesc(ctypes.Structure):
    _fields_ = [("a1", c_double * 2), ("a2", c_double * 2), ("order", c_int32), ("nbreak", c_int32),
                ("breakpoints", POINTER(c_double)), ("nq", c_int32), ("grid", c_int32 * 2),
                ("gset_kind", c_int32), ("mmax", c_int32 * 2), ("ecut", c_double), ("nk", c_int32),
                ("kfrac", POINTER(c_double)), ("nspecies", c_int32), ("species", POINTER(MbSpecies)),
                ("natoms", c_int32), ("atoms", POINTER(MbAtom))]


class MbWireDesc(ctypes.Structure):
    _fields_ = [("period", c_double), ("order", c_int32), ("nbreak_x", c_int32), ("breakpoints_x", POINTER(c_double)),
                ("nbreak_z", c_int32), ("breakpoints_z", POINTER(c_double)), ("nq", c_int32), ("ny", c_int32),
                ("ecut", c_double), ("nk", c_int32), ("kfrac", POINTER(c_double)), ("nspecies", c_int32),
                ("species", POINTER(MbSpecies)), ("natoms", c_int32), ("atoms", POINTER(MbAtom))]


class LanczosOpts(ctypes.Structure):
    _fields_ = [("block", c_int32), ("krylov", c_int32), ("krylov_global", c_int32), ("max_iter", c_int32),
                ("tol", c_double), ("sigma", c_double), ("switch_tol", c_double), ("seed", c_uint64),
                ("extra", c_int32), ("dense_low", c_int32)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("local_kernel", c_int32), ("lds_budget_kb", c_int32), ("plane_variant", c_int32),
                ("nl_matrix_cores", c_int32), ("combine_bands", c_int32), ("candidates", c_int32), ("local_ms", c_double),
                ("local_default_ms", c_double), ("nl_ms", c_double)]


class LanczosInfo(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("iters_low", c_int32), ("h_applies", c_int64), ("h_applies_low", c_int64),
                ("max_resid", c_double), ("time_ms", c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the in-tree library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libmbks.so not found at {path}; run `python -m paper_1406_4960_amd.build`")
    # torch bundles its own HIP runtime; load its libraries before this one so that
    # both runtimes are present before either initialises (the order that works)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp = c_void_p
    # initialise the library's HIP runtime before torch's bundled runtime does
    lib.mb_init.argtypes = [POINTER(c_int)]
    lib.mb_init.restype = c_int
    ndev = c_int(0)
    lib.mb_init(ctypes.byref(ndev))
    lib.ndevices = ndev.value
    lib.mb_problem_create.argtypes = [POINTER(MbDesc), c_int, POINTER(vp)]
    lib.mb_problem_destroy.argtypes = [vp]
    lib.mb_problem_dims.argtypes = [vp, c_int] + [POINTER(c_int64)] * 5
    lib.mb_problem_gvectors.argtypes = [vp, c_int, vp, vp]
    lib.mb_problem_zrule.argtypes = [vp, vp, vp]
    lib.mb_problem_zbands.argtypes = [vp, vp, vp]
    lib.mb_problem_projectors.argtypes = [vp, c_int, vp, vp, vp]
    lib.mb_problem_set_potential.argtypes = [vp, vp]
    for name in ("hpsi_apply", "hpsi_apply_gamma", "hpsi_apply_noalloc", "spsi_apply", "s_solve"):
        getattr(lib, name).argtypes = [vp, c_int, vp, vp, c_int64, c_int64, c_int, vp]
    lib.mb_lanczos_default_opts.argtypes = [POINTER(LanczosOpts)]
    lib.mb_lanczos_default_opts.restype = None
    lib.lanczos_lowest.argtypes = [vp, c_int, c_int, c_int, POINTER(LanczosOpts), vp, vp, vp,
                                   POINTER(LanczosInfo), vp]
    lib.mb_autotune.argtypes = [vp, c_int, c_int64, c_int, vp, POINTER(TuneInfo)]
    lib.mb_problem_reserve.argtypes = [vp, c_int, c_int64, c_int64, c_int]
    lib.mb_batch_create.argtypes = [vp, vp, c_int, POINTER(vp)]
    lib.mb_batch_destroy.argtypes = [vp]
    lib.hpsi_apply_batched.argtypes = [vp, vp, vp, vp, vp, c_int, vp]
    lib.lanczos_lowest_batched.argtypes = [vp, vp, c_int, POINTER(LanczosOpts), vp, vp, vp, vp]
    lib.mb_small_geneig.argtypes = [vp, vp, c_int, c_int, vp, vp, vp, vp]
    lib.mb_timer_enable.argtypes = [c_int]
    lib.mb_timer_read.argtypes = [c_int, POINTER(c_double), POINTER(c_int64), POINTER(c_int64)]
    lib.mb_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("mb_lanczos_default_opts", "mb_last_error"):
            getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise MbError(status, _lib.mb_last_error().decode())


def _prec(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


def _stream(stream):
    if stream is not None:
        return c_void_p(stream)
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(0)


STAGES = ("local", "nl_project", "combine", "spsi", "ssolve", "precond", "gram", "combo", "smalleig", "other",
          "local32", "density", "hartree")


def timer_enable(on: bool = True):
    _check(load().mb_timer_enable(int(on)))


def timer_read():
    """{stage: (total_ms, launches, units)} of the kernels recorded since timer_enable."""
    out = {}
    for k, name in enumerate(STAGES):
        ms, n, u = c_double(), c_int64(), c_int64()
        _check(load().mb_timer_read(k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(u)))
        out[name] = (ms.value, n.value, u.value)
    return out


def small_geneig(H: np.ndarray, S: np.ndarray, stream=None):
    """Batched projected eigenproblems on the GPU: H, S of shape (nz, N, N) complex.
    Returns (evals (nz, N), Y (nz, N, N), sweeps (nz,))."""
    H = np.ascontiguousarray(H, dtype=np.complex128)
    S = np.ascontiguousarray(S, dtype=np.complex128)
    nz, N, _ = H.shape
    ev = np.zeros((nz, N))
    Y = np.zeros((nz, N, N), dtype=np.complex128)
    sw = np.zeros(nz, dtype=np.int32)
    _check(load().mb_small_geneig(c_void_p(H.ctypes.data), c_void_p(S.ctypes.data), N, nz,
                                  c_void_p(ev.ctypes.data), c_void_p(Y.ctypes.data), c_void_p(sw.ctypes.data),
                                  _stream(stream)))
    return ev, Y, sw


def _species_atoms(desc):
    sp_arr = (MbSpecies * max(1, len(desc["species"])))()
    for n, sp in enumerate(desc["species"]):
        g = sp.get("gauss", [])
        if len(g) > MB_MAX_GAUSS:
            raise ValueError("too many Gaussian terms")
        sp_arr[n].ngauss = len(g)
        for t, (A, w) in enumerate(g):
            sp_arr[n].gauss_A[t] = A
            sp_arr[n].gauss_w[t] = w
        nl = bool(sp.get("nonlocal", False))
        sp_arr[n].nonlocal_ = int(nl)
        if nl:
            sp_arr[n].alpha_s = sp["alpha_s"]
            sp_arr[n].alpha_p = sp["alpha_p"]
            sp_arr[n].E_s = sp["E_s"]
            sp_arr[n].E_p = sp["E_p"]
            sp_arr[n].q_s = sp.get("q_s", 0.0)
            sp_arr[n].q_p = sp.get("q_p", 0.0)
    at_arr = (MbAtom * max(1, len(desc["atoms"])))()
    for n, at in enumerate(desc["atoms"]):
        at_arr[n].species = at["species"]
        for c in range(3):
            at_arr[n].pos[c] = at["pos"][c]
    return sp_arr, at_arr


class Problem:
    """Handle of one problem description; device=None builds host tables only."""

    def __init__(self, desc: dict, device: int | None = 0):
        """desc: a slab description, or a 1D-periodic one (desc["kind"] == "wire": keys
        period, order, breakpoints_x, breakpoints_z, nq, ny, ecut, kpts (fractions of
        2 pi / L), species, atoms)."""
        lib = load()
        self.desc = desc
        self.wire = desc.get("kind") == "wire"
        sp_arr, at_arr = _species_atoms(desc)
        if self.wire:
            bx = np.ascontiguousarray(desc["breakpoints_x"], dtype=np.float64)
            bz = np.ascontiguousarray(desc["breakpoints_z"], dtype=np.float64)
            kf = np.ascontiguousarray(np.array(desc["kpts"], dtype=np.float64).reshape(-1))
            w = MbWireDesc()
            w.period = desc["period"]
            w.order = desc["order"]
            w.nbreak_x = len(bx)
            w.breakpoints_x = bx.ctypes.data_as(POINTER(c_double))
            w.nbreak_z = len(bz)
            w.breakpoints_z = bz.ctypes.data_as(POINTER(c_double))
            w.nq = desc["nq"]
            w.ny = desc["ny"]
            w.ecut = desc["ecut"]
            w.nk = len(kf)
            w.kfrac = kf.ctypes.data_as(POINTER(c_double))
            w.nspecies = len(desc["species"])
            w.species = sp_arr
            w.natoms = len(desc["atoms"])
            w.atoms = at_arr
            h = c_void_p()
            _check(lib.mb_wire_create(ctypes.byref(w), -1 if device is None else int(device), ctypes.byref(h)))
            self.h = h
            self.device = device
            self.nk = len(kf)
            return
        bp = np.ascontiguousarray(desc["breakpoints"], dtype=np.float64)
        kf = np.ascontiguousarray(np.array(desc["kpts"], dtype=np.float64).reshape(-1, 2))
        d = MbDesc()
        d.a1[:] = list(desc["a1"])
        d.a2[:] = list(desc["a2"])
        d.order = desc["order"]
        d.nbreak = len(bp)
        d.breakpoints = bp.ctypes.data_as(POINTER(c_double))
        d.nq = desc["nq"]
        d.grid[:] = list(desc["grid"])
        rule = desc["gset"]
        if rule["kind"] == "box":
            d.gset_kind = 0
            d.mmax[:] = list(rule["mmax"])
        else:
            d.gset_kind = 1
            d.ecut = rule["ecut"]
        d.nk = len(kf)
        d.kfrac = kf.ctypes.data_as(POINTER(c_double))
        d.nspecies = len(desc["species"])
        d.species = sp_arr
        d.natoms = len(desc["atoms"])
        d.atoms = at_arr
        h = c_void_p()
        _check(lib.mb_problem_create(ctypes.byref(d), -1 if device is None else int(device), ctypes.byref(h)))
        self.h = h
        self.device = device
        self.nk = len(kf)

    def wire_dims(self):
        """Sizes of a 1D-periodic problem: splines along x and z, Gauss points along x and z, ny."""
        v = [c_int64() for _ in range(5)]
        _check(load().mb_wire_dims(self.h, *[ctypes.byref(x) for x in v]))
        nbx, nbz, nxq, nzq, ny = (x.value for x in v)
        return {"nbx": nbx, "nbz": nbz, "nxq": nxq, "nzq": nzq, "ny": ny}

    def close(self):
        if getattr(self, "h", None):
            load().mb_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # --- queries -------------------------------------------------------------
    def dims(self, ik: int = 0):
        v = [c_int64() for _ in range(5)]
        _check(load().mb_problem_dims(self.h, ik, *[ctypes.byref(x) for x in v]))
        ng, nb, ld, npj, nzq = (x.value for x in v)
        return {"ng": ng, "nb": nb, "ld": ld, "np": npj, "nzq": nzq}

    def gvectors(self, ik: int = 0):
        dm = self.dims(ik)
        m = np.zeros((dm["ng"], 2), dtype=np.int32)
        kg2 = np.zeros(dm["ng"])
        _check(load().mb_problem_gvectors(self.h, ik, c_void_p(m.ctypes.data), c_void_p(kg2.ctypes.data)))
        return m, kg2

    def zrule(self):
        n = self.dims(0)["nzq"]
        zq = np.zeros(n)
        wq = np.zeros(n)
        _check(load().mb_problem_zrule(self.h, c_void_p(zq.ctypes.data), c_void_p(wq.ctypes.data)))
        return zq, wq

    def zbands(self):
        nb = self.dims(0)["nb"]
        k = self.desc["order"]
        s = np.zeros((nb, k))
        d = np.zeros((nb, k))
        _check(load().mb_problem_zbands(self.h, c_void_p(s.ctypes.data), c_void_p(d.ctypes.data)))
        return s, d

    def projectors(self, ik: int = 0):
        dm = self.dims(ik)
        F = np.zeros((dm["np"], dm["ng"]), dtype=np.complex128)
        Z = np.zeros((dm["np"], dm["nb"]))
        E = np.zeros(dm["np"])
        _check(load().mb_problem_projectors(self.h, ik, c_void_p(F.ctypes.data), c_void_p(Z.ctypes.data),
                                            c_void_p(E.ctypes.data)))
        return F, Z, E

    def augmentation(self):
        """Augmentation charge q_p of every projector (zeros: norm-conserving)."""
        q = np.zeros(self.dims(0)["np"])
        _check(load().mb_problem_augmentation(self.h, c_void_p(q.ctypes.data)))
        return q

    def set_potential(self, v: np.ndarray):
        v = np.ascontiguousarray(v, dtype=np.float64)
        _check(load().mb_problem_set_potential(self.h, c_void_p(v.ctypes.data)))

    # --- operators -----------------------------------------------------------
    def _vec_args(self, ik, c, y, prec):
        nbands, nb, ld = c.shape
        return nbands, ld

    def hpsi(self, ik, c, y, prec="fp64", stream=None):
        nbands, ld = self._vec_args(ik, c, y, prec)
        _check(load().hpsi_apply(self.h, ik, _ptr(c), _ptr(y), nbands, ld, _prec(prec), _stream(stream)))

    def hpsi_gamma(self, ik, c, y, prec="fp64", stream=None):
        """y = H c for real wavefunctions at Gamma (c(-G) = conj c(G) in every band)."""
        nbands, ld = self._vec_args(ik, c, y, prec)
        _check(load().hpsi_apply_gamma(self.h, ik, _ptr(c), _ptr(y), nbands, ld, _prec(prec), _stream(stream)))

    def hpsi_noalloc(self, ik, c, y, prec="fp64", stream=None):
        nbands, ld = self._vec_args(ik, c, y, prec)
        _check(load().hpsi_apply_noalloc(self.h, ik, _ptr(c), _ptr(y), nbands, ld, _prec(prec), _stream(stream)))

    def spsi(self, ik, c, y, prec="fp64", stream=None):
        nbands, ld = self._vec_args(ik, c, y, prec)
        _check(load().spsi_apply(self.h, ik, _ptr(c), _ptr(y), nbands, ld, _prec(prec), _stream(stream)))

    def s_solve(self, ik, r, x, prec="fp64", stream=None):
        nbands, ld = self._vec_args(ik, r, x, prec)
        _check(load().s_solve(self.h, ik, _ptr(r), _ptr(x), nbands, ld, _prec(prec), _stream(stream)))

    def density(self, ik, c, w, rho, prec="fp64", stream=None):
        """rho += sum_b w[b] |phi_b|^2 at the Gauss planes: c [nbands][N_b][ld] (device),
        w [nbands] float64 (device), rho [N_q][N1][N2] float64 (device)."""
        nbands, nb, ld = c.shape
        _check(load().density_accumulate(self.h, ik, _ptr(c), ctypes.c_int64(nbands), ctypes.c_int64(ld), _ptr(w),
                                         _ptr(rho), _prec(prec), _stream(stream)))

    def hartree(self, rho, vh, vzg=None, stream=None):
        """vh = Hartree potential of rho on the grid at the Gauss planes ([N_q][N1][N2] float64,
        device); vzg (optional, [N_q][N1][N2] complex128): V(z_q, g) by grid frequency."""
        _check(load().hartree_potential(self.h, _ptr(rho), _ptr(vh), _ptr(vzg), _stream(stream)))

    def reserve(self, ik, max_bands, ld=0, lock=True):
        """Size the k-point's H work buffers for max_bands vectors and (lock) keep them fixed."""
        _check(load().mb_problem_reserve(self.h, ik, int(max_bands), int(ld), int(bool(lock))))

    def autotune(self, ik, nbands, prec="fp64", stream=None):
        """Measure the kernel choices for (ik, nbands, prec) and keep the fastest."""
        info = TuneInfo()
        _check(load().mb_autotune(self.h, ik, int(nbands), _prec(prec), _stream(stream), ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in TuneInfo._fields_}

    def tune_get(self, ik, prec="fp32"):
        """The kernel choices of k-point ik for a precision class (timing fields zero)."""
        info = TuneInfo()
        _check(load().mb_tune_get(self.h, ik, _prec(prec), ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in TuneInfo._fields_}

    def tune_set(self, ik, prec="fp32", **choices):
        """Apply kernel choices (keys of TuneInfo) to k-point ik without timing."""
        info = TuneInfo()
        cur = self.tune_get(ik, prec)
        cur.update(choices)
        for f, _ in TuneInfo._fields_:
            setattr(info, f, cur[f])
        _check(load().mb_tune_set(self.h, ik, _prec(prec), ctypes.byref(info)))

    def tune_save(self, path):
        """Merge this problem's tuned choices into the JSON cache file at path."""
        _check(load().mb_tune_save(self.h, os.fsencode(path)))

    def tune_load(self, path) -> int:
        """Apply the matching entries of the JSON cache file; returns how many applied."""
        n = ctypes.c_int(0)
        _check(load().mb_tune_load(self.h, os.fsencode(path), ctypes.byref(n)))
        return n.value

    @staticmethod
    def default_opts() -> LanczosOpts:
        o = LanczosOpts()
        load().mb_lanczos_default_opts(ctypes.byref(o))
        return o

    def lanczos_lowest(self, ik, nev, prec="fp64", opts=None, x0=None, x=None, stream=None,
                       raise_not_converged=True):
        """Returns (eig numpy array, x torch tensor [nev][nb][ld] complex128, info dict, status)."""
        import torch
        dm = self.dims(ik)
        if x is None:
            x = torch.zeros((nev, dm["nb"], dm["ld"]), dtype=torch.complex128, device=f"cuda:{self.device}")
        eig = np.zeros(nev)
        info = LanczosInfo()
        o = opts if opts is not None else self.default_opts()
        st = load().lanczos_lowest(self.h, ik, nev, _prec(prec), ctypes.byref(o), _ptr(x0),
                                   c_void_p(eig.ctypes.data), _ptr(x), ctypes.byref(info), _stream(stream))
        if st != 0 and not (st == -3 and not raise_not_converged):
            _check(st)
        inf = {f: getattr(info, f) for f, _ in LanczosInfo._fields_}
        return eig, x, inf, st


class Batch:
    """A fixed list of (Problem, k-point) items applied or solved together."""

    def __init__(self, items):
        self.items = [(pr, int(ik)) for pr, ik in items]
        n = len(self.items)
        probs = (c_void_p * n)(*[pr.h for pr, _ in self.items])
        iks = (c_int * n)(*[ik for _, ik in self.items])
        h = c_void_p()
        _check(load().mb_batch_create(ctypes.cast(probs, c_void_p), ctypes.cast(iks, c_void_p), n,
                                      ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().mb_batch_destroy(self.h)
            self.h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def hpsi(self, cs, ys, prec="fp64", stream=None):
        """ys[t] = H_t cs[t]; tensors [nbands_t][N_b][ld_t] (None or 0 bands: skipped)."""
        n = len(self.items)
        if len(cs) != n or len(ys) != n:
            raise ValueError("one input and one output block per item")
        cp = (c_void_p * n)(*[c.data_ptr() if c is not None else 0 for c in cs])
        yp = (c_void_p * n)(*[y.data_ptr() if y is not None else 0 for y in ys])
        nb = (c_int64 * n)(*[c.shape[0] if c is not None else 0 for c in cs])
        ld = (c_int64 * n)(*[c.shape[2] if c is not None else self.items[t][0].dims(self.items[t][1])["ld"]
                             for t, c in enumerate(cs)])
        _check(load().hpsi_apply_batched(self.h, ctypes.cast(cp, c_void_p), ctypes.cast(yp, c_void_p),
                                         ctypes.cast(nb, c_void_p), ctypes.cast(ld, c_void_p), _prec(prec),
                                         _stream(stream)))

    def bind(self, cs, ys, prec="fp64"):
        """Bind the blocks cs -> ys for hpsi_bound (repeatable and capturable)."""
        n = len(self.items)
        if len(cs) != n or len(ys) != n:
            raise ValueError("one input and one output block per item")
        cp = (c_void_p * n)(*[c.data_ptr() if c is not None else 0 for c in cs])
        yp = (c_void_p * n)(*[y.data_ptr() if y is not None else 0 for y in ys])
        nb = (c_int64 * n)(*[c.shape[0] if c is not None else 0 for c in cs])
        ld = (c_int64 * n)(*[c.shape[2] if c is not None else self.items[t][0].dims(self.items[t][1])["ld"]
                             for t, c in enumerate(cs)])
        _check(load().mb_batch_bind(self.h, ctypes.cast(cp, c_void_p), ctypes.cast(yp, c_void_p),
                                    ctypes.cast(nb, c_void_p), ctypes.cast(ld, c_void_p), _prec(prec)))
        self._bound = (cs, ys)  # keep the tensors alive while bound

    def hpsi_bound(self, stream=None):
        """H applied to the bound blocks (no allocation, no host synchronisation)."""
        _check(load().hpsi_apply_batched_bound(self.h, _stream(stream)))

    def lanczos_lowest(self, nev, prec="fp64", opts=None, stream=None, raise_not_converged=True):
        """nev: list of eigenpair counts per item.  Returns (eigs list, xs list of torch tensors,
        infos list of dicts, status)."""
        import torch
        n = len(self.items)
        eigs, xs = [], []
        for (pr, ik), k in zip(self.items, nev):
            dm = pr.dims(ik)
            eigs.append(np.zeros(max(k, 1)))
            xs.append(torch.zeros((max(k, 1), dm["nb"], dm["ld"]), dtype=torch.complex128,
                                  device=f"cuda:{pr.device}"))
        ne = (c_int * n)(*[int(k) for k in nev])
        ep = (c_void_p * n)(*[e.ctypes.data for e in eigs])
        xp = (c_void_p * n)(*[x.data_ptr() for x in xs])
        infos = (LanczosInfo * n)()
        o = opts if opts is not None else Problem.default_opts()
        st = load().lanczos_lowest_batched(self.h, ctypes.cast(ne, c_void_p), _prec(prec), ctypes.byref(o),
                                           ctypes.cast(ep, c_void_p), ctypes.cast(xp, c_void_p),
                                           ctypes.cast(infos, c_void_p), _stream(stream))
        if st != 0 and not (st == -3 and not raise_not_converged):
            _check(st)
        inf = [{f: getattr(infos[t], f) for f, _ in LanczosInfo._fields_} for t in range(n)]
        return [e[:k] for e, k in zip(eigs, nev)], [x[:k] for x, k in zip(xs, nev)], inf, st
