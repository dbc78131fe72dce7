"""Thin ctypes binding of libxfft.so (the C ABI of include/xfft.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Importing this module on a machine without the built library raises; there is
no fallback path.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxfft.so")

XFFT_OK, XFFT_NOT_CONVERGED = 0, 1
XFFT_EINVAL, XFFT_ENOMEM, XFFT_EDEVICE, XFFT_EBREAKDOWN = -1, -2, -3, -4
XFFT_FP64, XFFT_MIXED, XFFT_FP32 = 0, 1, 2

_PREC = {"fp64": XFFT_FP64, "mixed": XFFT_MIXED, "fp32": XFFT_FP32}
_SCHEME = {"lcg": 0, "nlcg": 1, "bb": 2, "basic": 3}


class XfftError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {_lib().xfft_strerror(code).decode()} (code {code})")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("rtol", ctypes.c_double),
        ("maxit", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("snap_eps", ctypes.c_double),
        ("d0_scale", ctypes.c_double),
        ("inner_rtol", ctypes.c_double),
        ("batch", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("scheme", ctypes.c_int32),
        ("discretization", ctypes.c_int32),
        ("voxel_matrices", ctypes.c_int32),
        ("warm_start", ctypes.c_int32),
        ("fft_variant", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.POINTER(ctypes.c_int32)),
        ("outer_iters", ctypes.POINTER(ctypes.c_int32)),
        ("final_res", ctypes.POINTER(ctypes.c_double)),
        ("seconds_setup", ctypes.c_double),
        ("seconds_solve", ctypes.c_double),
        ("n_enriched", ctypes.c_int64),
        ("n_irregular_voxels", ctypes.c_int64),
        ("n_cut_elements", ctypes.c_int64),
        ("n_multilabel", ctypes.c_int64),
        ("voxel_matrices", ctypes.c_int32),
        ("fft_variant", ctypes.c_int32),
    ]


EXPORTS = [
    "xfft_default_options", "xfft_setup", "xfft_solve", "xfft_solve_device", "xfft_set_lame",
    "xfft_grad_lame", "xfft_batch_solve", "xfft_apply_operator", "xfft_apply_precond", "xfft_voxel_stress",
    "xfft_apply_operator_noalloc", "xfft_get_layout", "xfft_profile", "xfft_profile_begin", "xfft_profile_end",
    "xfft_destroy",
    "xfft_strerror",
]

KERNEL_CLASSES = ["irregular_voxels", "regular_voxels", "enriched_gather", "fft_x_forward", "fft_y_forward",
                  "fft_z_green", "fft_y_inverse", "fft_x_inverse", "enriched_residual", "enriched_update",
                  "scalars"]

_LIB = None


def _lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_02172_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname.  Loading it first
    # makes the library bind to that instance, so that one HIP runtime serves
    # the process and torch device buffers and streams can be passed to the
    # C ABI; loaded the other way round, two runtimes would compete for the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, D, I32, I64, V = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p)
    lib.xfft_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.xfft_default_options.restype = None
    lib.xfft_setup.argtypes = [I32, D, D, I32, ctypes.c_int32, D, ctypes.POINTER(Options), ctypes.POINTER(P)]
    lib.xfft_setup.restype = ctypes.c_int
    lib.xfft_solve.argtypes = [P, ctypes.c_int32, D, D, D, D, D, ctypes.POINTER(Stats)]
    lib.xfft_solve.restype = ctypes.c_int
    lib.xfft_solve_device.argtypes = [P, ctypes.c_int32, V, V, V, V, ctypes.POINTER(Stats)]
    lib.xfft_solve_device.restype = ctypes.c_int
    lib.xfft_set_lame.argtypes = [P, D]
    lib.xfft_set_lame.restype = ctypes.c_int
    lib.xfft_grad_lame.argtypes = [P, D, D, D]
    lib.xfft_grad_lame.restype = ctypes.c_int
    lib.xfft_batch_solve.argtypes = [ctypes.POINTER(P), ctypes.c_int32, D, ctypes.POINTER(Stats)]
    lib.xfft_batch_solve.restype = ctypes.c_int
    lib.xfft_apply_operator.argtypes = [P, ctypes.c_int32, D, D, D, D]
    lib.xfft_apply_operator.restype = ctypes.c_int
    lib.xfft_apply_precond.argtypes = [P, ctypes.c_int32, D, D, D]
    lib.xfft_apply_precond.restype = ctypes.c_int
    lib.xfft_apply_operator_noalloc.argtypes = [P, V, V, V, V, V]
    lib.xfft_apply_operator_noalloc.restype = ctypes.c_int
    lib.xfft_voxel_stress.argtypes = [P, D, D, D]
    lib.xfft_voxel_stress.restype = ctypes.c_int
    lib.xfft_get_layout.argtypes = [P, I64, I64, D]
    lib.xfft_get_layout.restype = ctypes.c_int
    lib.xfft_profile.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, D, I32]
    lib.xfft_profile.restype = ctypes.c_int
    lib.xfft_profile_begin.argtypes = [P]
    lib.xfft_profile_begin.restype = ctypes.c_int
    lib.xfft_profile_end.argtypes = [P, D, I32]
    lib.xfft_profile_end.restype = ctypes.c_int
    lib.xfft_destroy.argtypes = [P]
    lib.xfft_destroy.restype = None
    lib.xfft_strerror.argtypes = [ctypes.c_int]
    lib.xfft_strerror.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if a is not None else None


def _check(rc, what, allow_not_converged=False):
    if rc == XFFT_OK or (allow_not_converged and rc == XFFT_NOT_CONVERGED):
        return rc
    raise XfftError(rc, what)


def default_options():
    o = Options()
    _lib().xfft_default_options(ctypes.byref(o))
    return o


class Problem:
    """One periodic cell: grid, nodal level set, nodal phase labels, Lame pairs."""

    def __init__(self, n, length, levelset, phase, lame, *, rtol=1e-10, maxit=20000, precision="fp64",
                 snap_eps=1e-6, d0_scale=1.0, inner_rtol=1e-6, batch=True, device=0, check_every=8,
                 use_graph=True, autotune=True, stream=None, scheme="lcg", discretization="xfem",
                 voxel_matrices="auto", warm_start=False, fft_variant="auto"):
        lib = _lib()
        self._h = None
        n = np.ascontiguousarray(n, dtype=np.int32)
        length = np.ascontiguousarray(length, dtype=np.float64)
        L = np.ascontiguousarray(levelset, dtype=np.float64).ravel()
        ph = np.ascontiguousarray(phase, dtype=np.int32).ravel()
        lame = np.ascontiguousarray(lame, dtype=np.float64).reshape(-1, 2)
        self.n = tuple(int(v) for v in n)
        self.N = int(np.prod(self.n))
        if L.size != self.N or ph.size != self.N:
            raise ValueError("levelset and phase must have n0*n1*n2 entries")
        self.nphase = lame.shape[0]
        o = default_options()
        o.rtol, o.maxit, o.precision = rtol, maxit, _PREC[precision]
        o.snap_eps, o.d0_scale, o.inner_rtol = snap_eps, d0_scale, inner_rtol
        o.batch, o.device, o.check_every = int(bool(batch)), device, check_every
        o.use_graph, o.autotune = int(bool(use_graph)), int(bool(autotune))
        o.stream = stream
        o.scheme = _SCHEME[scheme]
        o.discretization = {"xfem": 0, "p1": 1}[discretization]
        o.voxel_matrices = {"auto": -1, "never": 0, "always": 1}[voxel_matrices]
        o.warm_start = int(bool(warm_start))
        o.fft_variant = -1 if fft_variant == "auto" else int(fft_variant)
        h = ctypes.c_void_p()
        _check(lib.xfft_setup(_ip(n), _dp(length), _dp(L), _ip(ph), self.nphase, _dp(lame), ctypes.byref(o),
                              ctypes.byref(h)), "xfft_setup")
        self._h = h
        # counts solves and moduli changes: the stored unit-load solutions that
        # grad_lame uses belong to the current generation only
        self.generation = 0
        info = self.layout(with_arrays=False)
        self.nX = info["nX"]

    def close(self):
        if self._h is not None and self._h.value:
            _lib().xfft_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------ solve
    def solve(self, macro_strain, *, disp=False, stress=False, c_eff=False):
        E = np.ascontiguousarray(np.atleast_2d(macro_strain), dtype=np.float64)
        nl = E.shape[0]
        out = {}
        d = np.zeros((nl, 3, self.N)) if disp else None
        s = np.zeros((nl, 6, self.N)) if stress else None
        avg = np.zeros((nl, 6))
        C = np.zeros((6, 6)) if c_eff else None
        iters = np.zeros(nl, dtype=np.int32)
        outer = np.zeros(nl, dtype=np.int32)
        res = np.zeros(nl)
        st = Stats()
        st.iters = _ip(iters)
        st.outer_iters = _ip(outer)
        st.final_res = _dp(res)
        self.generation += 1
        rc = _lib().xfft_solve(self._h, nl, _dp(E), _dp(d), _dp(s), _dp(avg), _dp(C), ctypes.byref(st))
        _check(rc, "xfft_solve", allow_not_converged=True)
        out.update(avg_stress=avg, iters=iters, outer_iters=outer, final_res=res, converged=(rc == XFFT_OK),
                   seconds_setup=st.seconds_setup, seconds_solve=st.seconds_solve,
                   n_enriched=st.n_enriched, n_irregular_voxels=st.n_irregular_voxels,
                   n_cut_elements=st.n_cut_elements, n_multilabel=st.n_multilabel,
                   voxel_matrices=bool(st.voxel_matrices), fft_variant=int(st.fft_variant))
        if disp:
            out["disp"] = d
        if stress:
            out["stress"] = s
        if c_eff:
            out["c_eff"] = C
        return out

    def effective_stiffness(self):
        r = self.solve(np.eye(6), c_eff=True)
        return r["c_eff"], r

    def solve_device(self, strain_dev_ptr, nload, disp_dev_ptr=None, avg_dev_ptr=None, stream=None):
        """Device-pointer variant (pointers as ints, e.g. torch tensor.data_ptr())."""
        st = Stats()
        self.generation += 1
        rc = _lib().xfft_solve_device(self._h, nload, ctypes.c_void_p(strain_dev_ptr),
                                      ctypes.c_void_p(disp_dev_ptr) if disp_dev_ptr else None,
                                      ctypes.c_void_p(avg_dev_ptr) if avg_dev_ptr else None,
                                      ctypes.c_void_p(stream) if stream else None, ctypes.byref(st))
        return _check(rc, "xfft_solve_device", allow_not_converged=True)

    def set_lame(self, lame):
        lame = np.ascontiguousarray(lame, dtype=np.float64).reshape(-1, 2)
        if lame.shape[0] != self.nphase:
            raise ValueError("wrong number of phases")
        self.generation += 1
        _check(_lib().xfft_set_lame(self._h, _dp(lame)), "xfft_set_lame")

    def grad_lame(self, dL_dC):
        W = np.ascontiguousarray(dL_dC, dtype=np.float64).reshape(6, 6)
        g = np.zeros((self.nphase, 2))
        dC = np.zeros((self.nphase, 2, 6, 6))
        _check(_lib().xfft_grad_lame(self._h, _dp(W), _dp(g), _dp(dC)), "xfft_grad_lame")
        return g, dC

    # ------------------------------------------------------------------ step level
    def apply_operator(self, x, macro_strain=None, precision="fp64", with_stress=True):
        """y = r(x) and <sigma>; with_stress=False runs the stress-free kernels of the CG
        iterations and returns avg = None."""
        x = np.ascontiguousarray(x, dtype=np.float64).ravel()
        if x.size != 3 * (self.N + self.nX):
            raise ValueError("x must have 3 (N + nX) entries")
        y = np.zeros_like(x)
        avg = np.zeros(6) if with_stress else None
        E = None if macro_strain is None else np.ascontiguousarray(macro_strain, dtype=np.float64)
        _check(_lib().xfft_apply_operator(self._h, _PREC[precision], _dp(x), _dp(E), _dp(y), _dp(avg)),
               "xfft_apply_operator")
        return y, avg

    def apply_operator_noalloc(self, x_dev_ptr, y_dev_ptr, macro_strain_dev_ptr=None, avg_dev_ptr=None,
                               stream=None):
        """xfft_apply_operator_noalloc on device pointers (ints, e.g. tensor.data_ptr()); FP64.

        Enqueued on ``stream`` (or the problem's stream) without waiting for it."""
        vp = lambda v: ctypes.c_void_p(v) if v else None
        rc = _lib().xfft_apply_operator_noalloc(self._h, vp(x_dev_ptr), vp(macro_strain_dev_ptr), vp(y_dev_ptr),
                                                vp(avg_dev_ptr), vp(stream))
        return _check(rc, "xfft_apply_operator_noalloc")

    def voxel_stress(self, x, macro_strain=None):
        """Voxel-average Mandel stress (6, N) of the state x (FP64)."""
        x = np.ascontiguousarray(x, dtype=np.float64).ravel()
        if x.size != 3 * (self.N + self.nX):
            raise ValueError("x must have 3 (N + nX) entries")
        out = np.zeros((6, self.N))
        E = None if macro_strain is None else np.ascontiguousarray(macro_strain, dtype=np.float64)
        _check(_lib().xfft_voxel_stress(self._h, _dp(x), _dp(E), _dp(out)), "xfft_voxel_stress")
        return out

    def apply_precond(self, f, precision="fp64"):
        f = np.ascontiguousarray(f, dtype=np.float64).ravel()
        if f.size != 3 * (self.N + self.nX):
            raise ValueError("f must have 3 (N + nX) entries")
        y = np.zeros_like(f)
        r2 = np.zeros(1)
        _check(_lib().xfft_apply_precond(self._h, _PREC[precision], _dp(f), _dp(y), _dp(r2)), "xfft_apply_precond")
        return y, float(r2[0])

    def profile(self, precision="fp32", nrhs=6, nrep=10):
        """Average per-launch kernel times (ms) of one CG iteration, by kernel class."""
        ms = np.zeros(len(KERNEL_CLASSES))
        cnt = np.zeros(len(KERNEL_CLASSES), dtype=np.int32)
        _check(_lib().xfft_profile(self._h, _PREC[precision], nrhs, nrep, _dp(ms), _ip(cnt)), "xfft_profile")
        return {k: (float(m), int(c)) for k, m, c in zip(KERNEL_CLASSES, ms, cnt)}

    def profile_begin(self):
        """Start timing every kernel launch (see profile_end)."""
        _check(_lib().xfft_profile_begin(self._h), "xfft_profile_begin")

    def profile_end(self):
        """Per kernel class and precision: (average ms per launch, launches) since profile_begin."""
        n = 2 * len(KERNEL_CLASSES)
        ms = np.zeros(n)
        cnt = np.zeros(n, dtype=np.int32)
        _check(_lib().xfft_profile_end(self._h, _dp(ms), _ip(cnt)), "xfft_profile_end")
        out = {}
        for i, (m, c) in enumerate(zip(ms, cnt)):
            prec = "fp32" if i < len(KERNEL_CLASSES) else "fp64"
            out[(KERNEL_CLASSES[i % len(KERNEL_CLASSES)], prec)] = (float(m), int(c))
        return out

    def layout(self, with_arrays=True):
        info = np.zeros(6, dtype=np.int64)
        _check(_lib().xfft_get_layout(self._h, info.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None, None),
               "xfft_get_layout")
        out = dict(N=int(info[0]), nX=int(info[1]), n_irregular_voxels=int(info[2]), n_cut_elements=int(info[3]),
                   n_multilabel=int(info[4]), nphase=int(info[5]))
        if with_arrays and out["nX"] > 0:
            jl = np.zeros(out["nX"], dtype=np.int64)
            d0 = np.zeros(out["nX"])
            _check(_lib().xfft_get_layout(self._h, info.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          jl.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(d0)),
                   "xfft_get_layout")
            out.update(jlist=jl, d0=d0)
        return out


def batch_effective_stiffness(problems, with_stats=False):
    """C_eff of several problems (uneven grids allowed): array (nprob, 6, 6)."""
    arr = (ctypes.c_void_p * len(problems))(*[p._h.value for p in problems])
    C = np.zeros((len(problems), 6, 6))
    iters = np.zeros((len(problems), 6), dtype=np.int32)
    outer = np.zeros((len(problems), 6), dtype=np.int32)
    st = (Stats * len(problems))()
    for p in problems:
        p.generation += 1
    for i in range(len(problems)):
        st[i].iters = iters[i].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        st[i].outer_iters = outer[i].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    rc = _lib().xfft_batch_solve(arr, len(problems), _dp(C), st)
    _check(rc, "xfft_batch_solve", allow_not_converged=True)
    if with_stats:
        return C, dict(iters=iters, outer_iters=outer, converged=(rc == XFFT_OK), seconds_solve=st[0].seconds_solve)
    return C
