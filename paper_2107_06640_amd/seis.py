"""Python binding of the C ABI in include/seis.h (argument marshalling only).

Every step of the element update runs in the HIP library libseis.so; this
module only converts numpy arrays to pointers and back. If the library is
missing the import of ``Solver`` fails: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SEIS_LIB", os.path.join(_HERE, "libseis.so"))

SEIS_FP64, SEIS_FP32, SEIS_BF16, SEIS_BF16_SPLIT = 0, 1, 2, 3
SEIS_KERNEL_TUNED, SEIS_KERNEL_PLAIN = 0, 1
# "bf16x3": split BF16 operands (hi + lo), three BF16 products per product
PRECISIONS = {"fp64": SEIS_FP64, "fp32": SEIS_FP32, "bf16": SEIS_BF16, "bf16x3": SEIS_BF16_SPLIT}
KERNELS = {"tuned": SEIS_KERNEL_TUNED, "plain": SEIS_KERNEL_PLAIN}
ERRORS = {-1: "SEIS_EINVAL", -2: "SEIS_ENOMEM", -3: "SEIS_EDEVICE", -4: "SEIS_EORDER", -5: "SEIS_ERANGE"}

EXPORTED = ["seis_default_options", "seis_setup", "seis_write", "seis_predict", "seis_correct", "seis_step",
            "seis_run", "seis_read", "seis_read_elements", "seis_info", "seis_cluster_of", "seis_sync",
            "seis_destroy", "seis_last_error", "seis_profile", "seis_profile_read", "seis_energy",
            "seis_energy_noalloc", "seis_points", "seis_points_info", "seis_sample", "seis_set_uplift",
            "seis_set_fault", "seis_fault_read"]
FAULT_POINT_VALUES = 14  # x, y, z, slip (3), slip path, slip rate (3), shear traction (3), normal stress
SEIS_POINTS_SEA_SURFACE, SEIS_POINTS_SEAFLOOR = -1, -2


class SeisError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Mesh_t(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("xyz", C.POINTER(C.c_double)),
                ("n_elements", C.c_int64), ("tet", C.POINTER(C.c_int64)),
                ("face_kind", C.POINTER(C.c_int8)), ("period", C.c_double * 3)]


class Materials_t(C.Structure):
    _fields_ = [("rho", C.POINTER(C.c_double)), ("lam", C.POINTER(C.c_double)), ("mu", C.POINTER(C.c_double))]


class Options_t(C.Structure):
    _fields_ = [("precision", C.c_int), ("kernel", C.c_int), ("cfl", C.c_double), ("g", C.c_double),
                ("max_clusters", C.c_int), ("stream", C.c_void_p), ("tile", C.c_int), ("graph", C.c_int),
                ("mc_min", C.c_int), ("fused", C.c_int), ("acoustic", C.c_int)]


class Info_t(C.Structure):
    _fields_ = [("order", C.c_int), ("n_basis", C.c_int), ("n_face_nodes", C.c_int), ("n_eta_points", C.c_int),
                ("precision", C.c_int), ("kernel", C.c_int), ("n_clusters", C.c_int),
                ("n_elements", C.c_int64), ("n_gravity_faces", C.c_int64), ("dt_min", C.c_double),
                ("time", C.c_double), ("cluster_size", C.c_int64 * 16), ("updates_per_macro_step", C.c_int64),
                ("device_bytes", C.c_int64), ("launch", C.c_int * 8), ("launch_source", C.c_int),
                ("fused", C.c_int), ("shape", C.c_int), ("n_acoustic_groups", C.c_int64),
                ("n_fault_faces", C.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libseis.so and declare the signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run python -m paper_2107_06640_amd.build")
    # torch ships its own HIP runtime under the same soname as the one the
    # library links. Loading torch first makes the library bind to that one
    # runtime, so that torch's streams and device memory are valid in it;
    # loaded the other way round, the process would hold two runtimes and
    # torch's device initialisation fails.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    lib.seis_default_options.argtypes = [C.POINTER(Options_t)]
    lib.seis_default_options.restype = None
    lib.seis_setup.argtypes = [C.POINTER(Mesh_t), C.POINTER(Materials_t), C.c_int, C.POINTER(Options_t),
                               C.POINTER(P)]
    lib.seis_write.argtypes = [P, dp, dp]
    lib.seis_predict.argtypes = [P, C.c_int]
    lib.seis_correct.argtypes = [P, C.c_int]
    lib.seis_step.argtypes = [P]
    lib.seis_run.argtypes = [P, C.c_int]
    lib.seis_read.argtypes = [P, dp, dp]
    lib.seis_read_elements.argtypes = [P, C.POINTER(C.c_int64), C.c_int64, dp]
    lib.seis_info.argtypes = [P, C.POINTER(Info_t)]
    lib.seis_cluster_of.argtypes = [P, C.POINTER(C.c_int32)]
    lib.seis_sync.argtypes = [P]
    lib.seis_profile.argtypes = [P, C.c_int]
    lib.seis_profile_read.argtypes = [P, dp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.seis_energy.argtypes = [P, C.c_void_p]
    lib.seis_points.argtypes = [P, C.c_int64, dp, C.POINTER(C.c_int)]
    lib.seis_points_info.argtypes = [P, C.c_int, C.POINTER(C.c_int64), dp, C.POINTER(C.c_int64)]
    lib.seis_sample.argtypes = [P, C.c_int, C.c_void_p, C.c_void_p]
    lib.seis_set_uplift.argtypes = [P, C.c_int, dp]
    lib.seis_set_fault.argtypes = [P, C.c_int64, C.c_int, dp]
    lib.seis_fault_read.argtypes = [P, dp]
    lib.seis_energy_noalloc.argtypes = [P, C.c_void_p]
    lib.seis_destroy.argtypes = [P]
    lib.seis_destroy.restype = None
    lib.seis_last_error.argtypes = [P]
    lib.seis_last_error.restype = C.c_char_p
    for name in ("seis_setup", "seis_write", "seis_predict", "seis_correct", "seis_step", "seis_run",
                 "seis_read", "seis_read_elements", "seis_info", "seis_cluster_of", "seis_sync",
                 "seis_profile", "seis_profile_read", "seis_energy", "seis_energy_noalloc", "seis_points",
                 "seis_points_info", "seis_sample", "seis_set_uplift", "seis_set_fault", "seis_fault_read"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class Solver:
    """One library handle (seis_setup ... seis_destroy)."""

    def __init__(self, xyz, tet, face_kind, period, rho, lam, mu, order, *, precision="fp64",
                 kernel="tuned", cfl=0.35, g=9.81, max_clusters=1, stream=None, tile=0, graph=False,
                 mc_min=None, fused=True, acoustic=True):
        lib = load_library()
        self._lib = lib
        self._keep = [np.ascontiguousarray(xyz, dtype=np.float64), np.ascontiguousarray(tet, dtype=np.int64),
                      np.ascontiguousarray(face_kind, dtype=np.int8), np.ascontiguousarray(rho, dtype=np.float64),
                      np.ascontiguousarray(lam, dtype=np.float64), np.ascontiguousarray(mu, dtype=np.float64)]
        x, t, f, r, l, m = self._keep
        mesh = Mesh_t(x.shape[0], _ptr(x, C.c_double), t.shape[0], _ptr(t, C.c_int64), _ptr(f, C.c_int8),
                      (C.c_double * 3)(*[float(v) for v in period]))
        mats = Materials_t(_ptr(r, C.c_double), _ptr(l, C.c_double), _ptr(m, C.c_double))
        opt = Options_t()
        lib.seis_default_options(C.byref(opt))
        opt.precision = PRECISIONS[precision]
        opt.kernel = KERNELS[kernel]
        opt.cfl = cfl
        opt.g = g
        opt.max_clusters = max_clusters
        opt.stream = stream
        opt.tile = tile
        opt.graph = 1 if graph else 0
        if mc_min is not None:
            opt.mc_min = int(mc_min)
        opt.fused = 1 if fused else 0
        opt.acoustic = 1 if acoustic else 0
        h = C.c_void_p()
        rc = lib.seis_setup(C.byref(mesh), C.byref(mats), int(order), C.byref(opt), C.byref(h))
        if rc != 0:
            raise SeisError(rc, lib.seis_last_error(None).decode())
        self._h = h
        self._keep = None
        inf = self.info()
        self.E, self.B, self.nq = inf["n_elements"], inf["n_basis"], inf["n_eta_points"]
        self.n_gravity_faces = inf["n_gravity_faces"]

    def _check(self, rc):
        if rc != 0:
            raise SeisError(rc, self._lib.seis_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.seis_destroy(self._h)
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

    def write(self, dofs=None, eta=None):
        d = None if dofs is None else np.ascontiguousarray(dofs, dtype=np.float64)
        e = None if eta is None else np.ascontiguousarray(eta, dtype=np.float64)
        if d is not None and d.shape != (self.E, self.B, 9):
            raise ValueError(f"dofs must have shape {(self.E, self.B, 9)}")
        if e is not None and e.shape != (self.n_gravity_faces, self.nq):
            raise ValueError(f"eta must have shape {(self.n_gravity_faces, self.nq)}")
        self._check(self._lib.seis_write(self._h, None if d is None else _ptr(d, C.c_double),
                                         None if e is None else _ptr(e, C.c_double)))

    def set_uplift(self, sources):
        """Uplift history of the prescribed-velocity faces: sources [n][5] = (A, x, y, w, T)."""
        src = np.ascontiguousarray(sources, dtype=np.float64).reshape(-1, 5)
        self._check(self._lib.seis_set_uplift(self._h, src.shape[0], _ptr(src, C.c_double)))

    def set_fault(self, params, law=0):
        """Friction of the fault faces (one row for all, or one per face):
        law 0 (slip weakening): (s0, tau0_x, tau0_y, tau0_z, mu_s, mu_d, D_c, C);
        law 1 (rate and state): (s0, tau0_x, tau0_y, tau0_z, a, b, L, V0, f0, f_w, V_w, psi0)."""
        n = self.info()["n_fault_faces"]
        k = 8 if law == 0 else 12
        p = np.ascontiguousarray(np.broadcast_to(np.asarray(params, dtype=np.float64), (n, k)))
        self._check(self._lib.seis_set_fault(self._h, n, int(law), _ptr(p, C.c_double)))

    def fault_read(self):
        """Fault state [n_fault_faces][n_face_nodes][14] (see FAULT_POINT_VALUES)."""
        inf = self.info()
        out = np.zeros((inf["n_fault_faces"], inf["n_face_nodes"], FAULT_POINT_VALUES))
        self._check(self._lib.seis_fault_read(self._h, _ptr(out, C.c_double)))
        return out

    def predict(self, c):
        self._check(self._lib.seis_predict(self._h, int(c)))

    def correct(self, c):
        self._check(self._lib.seis_correct(self._h, int(c)))

    def step(self):
        self._check(self._lib.seis_step(self._h))

    def run(self, n):
        self._check(self._lib.seis_run(self._h, int(n)))

    def sync(self):
        self._check(self._lib.seis_sync(self._h))

    def read(self, dofs=True, eta=True):
        """(dofs [E][B][9], eta [F_g][(N+1)^2]) in FP64; a part not asked for is None."""
        d = np.empty((self.E, self.B, 9)) if dofs else None
        e = np.empty((self.n_gravity_faces, self.nq)) if eta else None
        self._check(self._lib.seis_read(self._h, None if d is None else _ptr(d, C.c_double),
                                        None if e is None else _ptr(e, C.c_double)))
        return d, e

    def read_elements(self, ids):
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        d = np.empty((ids.size, self.B, 9))
        self._check(self._lib.seis_read_elements(self._h, _ptr(ids, C.c_int64), ids.size, _ptr(d, C.c_double)))
        return d

    def profile(self, enable=True):
        self._check(self._lib.seis_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """Per-kernel totals: {'predict'|'gravity'|'correct'|'fault': (ms, launches, elements)}."""
        ms = np.zeros(4)
        la = np.zeros(4, dtype=np.int64)
        el = np.zeros(4, dtype=np.int64)
        self._check(self._lib.seis_profile_read(self._h, _ptr(ms, C.c_double), _ptr(la, C.c_int64),
                                                _ptr(el, C.c_int64)))
        return {k: (float(ms[i]), int(la[i]), int(el[i]))
                for i, k in enumerate(("predict", "gravity", "correct", "fault"))}

    def energy_into(self, out_ptr, noalloc=False):
        """Energy and field norms into 12 doubles at device address ``out_ptr`` (asynchronous)."""
        fn = self._lib.seis_energy_noalloc if noalloc else self._lib.seis_energy
        self._check(fn(self._h, C.c_void_p(int(out_ptr))))

    def points(self, xyz):
        """Define receivers at physical points [n, 3]; returns the set id."""
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        i = C.c_int()
        self._check(self._lib.seis_points(self._h, x.shape[0], _ptr(x, C.c_double), C.byref(i)))
        return i.value

    def points_info(self, set_id):
        """(points [n, 3], caller element ids [n]) of a point set."""
        n = C.c_int64()
        self._check(self._lib.seis_points_info(self._h, int(set_id), C.byref(n), None, None))
        x = np.empty((n.value, 3))
        e = np.empty(n.value, dtype=np.int64)
        self._check(self._lib.seis_points_info(self._h, int(set_id), None, _ptr(x, C.c_double), _ptr(e, C.c_int64)))
        return x, e

    def sample_into(self, set_id, out_ptr, eta_ptr=None):
        """The nine quantities at a set's points into device memory [n][9] (asynchronous)."""
        self._check(self._lib.seis_sample(self._h, int(set_id), C.c_void_p(int(out_ptr)),
                                          None if eta_ptr is None else C.c_void_p(int(eta_ptr))))

    def info(self):
        inf = Info_t()
        self._check(self._lib.seis_info(self._h, C.byref(inf)))
        out = {k: getattr(inf, k) for k, _ in Info_t._fields_}
        out["cluster_size"] = list(inf.cluster_size)[: inf.n_clusters]
        out["launch"] = list(inf.launch)
        return out

    def cluster_of(self):
        out = np.empty(self.E, dtype=np.int32)
        self._check(self._lib.seis_cluster_of(self._h, _ptr(out, C.c_int32)))
        return out


def from_mesh(mesh, mats, order, **kw) -> Solver:
    """Solver from an inputs.Mesh and (rho, lambda, mu)."""
    rho, lam, mu = mats
    return Solver(mesh.xyz, mesh.tet, mesh.face_kind, mesh.period, rho, lam, mu, order, **kw)
