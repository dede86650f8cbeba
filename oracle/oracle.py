"""ctypes front end of the FP64 C oracle (tlmpm_oracle.c).

Test infrastructure only.  Arrays cross the boundary as C-contiguous float64
array-of-structs ([n][3] positions, [n][9] row-major F); ternary codes are held as
one uint8 digit per cut.
"""
import ctypes as C
import os

import numpy as np

from .build import LIB, build

__all__ = ["Params", "Blade", "Tool", "OracleScene", "lib", "load", "shape", "neo_hookean_P",
           "neo_hookean_psi", "fcr_P", "fcr_psi", "polar", "visc_P", "vm_project", "conflict", "encode", "digit", "couple", "label_digit",
           "labels_on", "set_threads", "get_threads"]


class Params(C.Structure):
    _fields_ = [
        ("dx", C.c_double), ("origin", C.c_double * 3), ("cells", C.c_int32 * 3),
        ("max_cuts", C.c_int32), ("dt", C.c_double), ("gravity", C.c_double * 3),
        ("beta", C.c_double), ("nu", C.c_double),
        ("s_R", C.c_double), ("s_n", C.c_double), ("gamma_k", C.c_double),
        ("gamma_c", C.c_double), ("mu_s", C.c_double), ("mu_d", C.c_double),
        ("material_contact", C.c_int32), ("floor_on", C.c_int32), ("floor_z", C.c_double),
        ("G_c", C.c_double), ("zeta", C.c_double), ("u_min", C.c_double),
        ("single_field", C.c_int32), ("material", C.c_int32),
        ("viscosity", C.c_double), ("yield_stress", C.c_double), ("stencil", C.c_int32), ("pad_", C.c_int32),
    ]


class Blade(C.Structure):
    _fields_ = [
        ("cut_index", C.c_int32), ("new_cut", C.c_int32),
        ("x_e", C.c_double * 3), ("n", C.c_double * 3), ("e", C.c_double * 3),
        ("d", C.c_double * 3), ("v_e", C.c_double * 3),
        ("half_len", C.c_double), ("half_width", C.c_double),
        ("b_back", C.c_double), ("b_lead", C.c_double),
    ]


class Tool(C.Structure):
    _fields_ = [
        ("blade", Blade), ("x_B", C.c_double * 3), ("v_B", C.c_double * 3),
        ("omega_B", C.c_double * 3), ("w_B", C.c_double),
        ("contact", C.c_int32), ("cutting", C.c_int32),
        ("inv_mass", C.c_double), ("inv_inertia", C.c_double * 9),
    ]


_lib = None


def load(path):
    """Load a compiled oracle library from `path` and declare its entry points.
    lib() loads the one built from oracle/tlmpm_oracle.c; the pins also load
    variants built from edited copies of the source to show that each pin fails
    under the mistake it targets."""
    L = C.CDLL(path)
    _declare(L)
    return L


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = load(LIB)
    return _lib


def _declare(L):
    dp = C.POINTER(C.c_double)
    u8p = C.POINTER(C.c_uint8)
    L.orc_create.restype = C.c_void_p
    L.orc_create.argtypes = [C.POINTER(Params), C.c_long, dp, dp, dp, dp, dp]
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_assign_labels.restype = C.c_long
    L.orc_assign_labels.argtypes = [C.c_void_p, C.POINTER(Blade), C.c_int]
    L.orc_step.restype = C.c_int
    L.orc_step.argtypes = [C.c_void_p, C.POINTER(Tool), C.c_int, dp, C.c_int]
    L.orc_get.argtypes = [C.c_void_p, dp, dp, dp, u8p, dp]
    L.orc_set.argtypes = [C.c_void_p, dp, dp, dp, u8p, dp]
    L.orc_shape.restype = C.c_int
    L.orc_shape.argtypes = [C.POINTER(Params), dp, C.POINTER(C.c_long), dp, dp]
    L.orc_neo_hookean_P.restype = C.c_int
    L.orc_neo_hookean_P.argtypes = [C.c_double, C.c_double, dp, dp]
    L.orc_neo_hookean_psi.restype = C.c_double
    L.orc_neo_hookean_psi.argtypes = [C.c_double, C.c_double, dp]
    L.orc_fcr_P.restype = C.c_int
    L.orc_fcr_P.argtypes = [C.c_double, C.c_double, dp, dp]
    L.orc_fcr_psi.restype = C.c_double
    L.orc_fcr_psi.argtypes = [C.c_double, C.c_double, dp]
    L.orc_polar.restype = C.c_int
    L.orc_polar.argtypes = [dp, dp, dp]
    L.orc_vm_project.restype = C.c_int
    L.orc_vm_project.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
    L.orc_visc_P.restype = C.c_int
    L.orc_visc_P.argtypes = [C.c_double, dp, dp, dp]
    L.orc_conflict.restype = C.c_int
    L.orc_conflict.argtypes = [C.c_uint64, C.c_uint64, C.c_int]
    L.orc_encode.restype = C.c_uint64
    L.orc_encode.argtypes = [u8p, C.c_int]
    L.orc_digit.restype = C.c_int
    L.orc_digit.argtypes = [C.c_uint64, C.c_int]
    L.orc_couple.argtypes = [C.c_int, dp, C.POINTER(C.c_uint64), C.c_int, dp, dp]
    L.orc_label_digit.restype = C.c_int
    L.orc_label_digit.argtypes = [dp, dp, C.POINTER(Blade), C.c_double, C.c_int]
    L.orc_candidates.argtypes = [C.c_void_p, u8p]
    L.orc_label_pass.restype = C.c_long
    L.orc_label_pass.argtypes = [C.c_long, dp, dp, u8p, C.c_int, C.POINTER(Blade), C.c_int, C.c_double]
    L.orc_last_pairs.restype = C.c_long
    L.orc_last_pairs.argtypes = [C.c_void_p]
    L.orc_last_candidates.restype = C.c_long
    L.orc_last_candidates.argtypes = [C.c_void_p]
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_get_threads.restype = C.c_int
    L.orc_grid_dump.restype = C.c_long
    L.orc_grid_dump.argtypes = [C.c_void_p, C.c_long, C.POINTER(C.c_int64), C.POINTER(C.c_uint64),
                                dp, dp, dp, dp]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _vec3(dst, src):
    for i in range(3):
        dst[i] = float(src[i])


def make_blade(b):
    """Blade from a dict with keys cut_index, new_cut, x_e, n, e, d, v_e, half_len,
    half_width, b_back, b_lead.  Values are taken as given (float32 inputs widen
    exactly)."""
    B = Blade()
    B.cut_index = int(b["cut_index"])
    B.new_cut = int(b.get("new_cut", 0))
    for k in ("x_e", "n", "e", "d", "v_e"):
        _vec3(getattr(B, k), np.asarray(b[k], dtype=np.float64))
    for k in ("half_len", "half_width", "b_back", "b_lead"):
        setattr(B, k, float(b[k]))
    return B


def make_tool(t):
    T = Tool()
    T.blade = make_blade(t["blade"])
    for k in ("x_B", "v_B", "omega_B"):
        _vec3(getattr(T, k), np.asarray(t.get(k, (0.0, 0.0, 0.0)), dtype=np.float64))
    T.w_B = float(t.get("w_B", 0.0))
    T.inv_mass = float(t.get("inv_mass", 0.0))
    ii = np.asarray(t.get("inv_inertia", np.zeros(9)), dtype=np.float64).reshape(9)
    for i in range(9):
        T.inv_inertia[i] = float(ii[i])
    T.contact = int(t.get("contact", 1))
    T.cutting = int(t.get("cutting", 0))
    return T


def make_params(p):
    P = Params()
    P.dx = float(p["dx"])
    _vec3(P.origin, p["origin"])
    for i in range(3):
        P.cells[i] = int(p["cells"][i])
    P.max_cuts = int(p.get("max_cuts", 4))
    P.dt = float(p["dt"])
    _vec3(P.gravity, p.get("gravity", (0.0, 0.0, -9.81)))
    P.beta = float(p.get("flip_beta", 0.95))
    P.nu = float(p["nu"])
    for k in ("s_R", "s_n", "gamma_k", "gamma_c", "mu_s", "mu_d", "G_c", "zeta", "u_min", "floor_z"):
        setattr(P, k, float(p[k]))
    P.material_contact = int(p.get("material_contact", 0))
    P.floor_on = int(p.get("floor_on", 0))
    P.single_field = int(p.get("single_field", 0))
    P.material = int(p.get("material", 0))
    P.viscosity = float(p.get("viscosity", 0.0))
    P.yield_stress = float(p.get("yield_stress", 0.0))
    P.stencil = int(p.get("stencil", 0))
    return P


class OracleScene:
    """One FP64 scene.  ``scene`` is a dict as produced by the workload generators:
    params (dict) plus arrays X [n,3], v0 [n,3] or None, vol0 [n], mass [n], E [n]."""

    def __init__(self, scene, L=None):
        L = L or lib()
        self.L = L
        self.P = make_params(scene["params"])
        X = _f64(scene["X"], (-1, 3))
        self.n = X.shape[0]
        v0 = scene.get("v0")
        v0 = _f64(v0, (-1, 3)) if v0 is not None else None
        vol0 = _f64(np.broadcast_to(np.asarray(scene["vol0"], np.float64), (self.n,)))
        mass = _f64(np.broadcast_to(np.asarray(scene["mass"], np.float64), (self.n,)))
        E = _f64(np.broadcast_to(np.asarray(scene["E"], np.float64), (self.n,)))
        self._keep = (X, v0, vol0, mass, E)
        self.h = L.orc_create(C.byref(self.P), self.n, _dp(X), _dp(v0) if v0 is not None else None,
                              _dp(vol0), _dp(mass), _dp(E))
        if not self.h:
            raise ValueError("oracle scene rejected (particle outside the grid or bad parameters)")
        self.K = self.P.max_cuts

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None

    def assign_labels(self, blades):
        arr = (Blade * max(1, len(blades)))(*[make_blade(b) for b in blades])
        r = self.L.orc_assign_labels(self.h, arr, len(blades))
        if r < 0:
            raise ValueError("bad cut index")
        return r

    def step(self, tools=(), brute_pairs=False):
        """One substep; returns (status, wrench [n_tools, 6])."""
        nt = len(tools)
        arr = (Tool * max(1, nt))(*[make_tool(t) for t in tools])
        w = np.zeros((max(1, nt), 6))
        st = self.L.orc_step(self.h, arr, nt, _dp(w), int(bool(brute_pairs)))
        return st, w[:nt]

    def get(self):
        n, K = self.n, self.K
        x = np.empty((n, 3))
        v = np.empty((n, 3))
        F = np.empty((n, 3, 3))
        dig = np.zeros((n, max(1, K)), np.uint8)
        D = np.empty(n)
        self.L.orc_get(self.h, _dp(x), _dp(v), _dp(F), dig.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(D))
        return {"x": x, "v": v, "F": F, "digits": dig[:, :K], "D": D}

    def set(self, x=None, v=None, F=None, digits=None, D=None):
        n, K = self.n, self.K
        keep = []

        def conv(a, shape):
            if a is None:
                return None
            a = _f64(a, shape)
            keep.append(a)
            return _dp(a)

        dg = None
        if digits is not None:
            d = np.ascontiguousarray(np.asarray(digits, np.uint8).reshape(n, K))
            keep.append(d)
            dg = d.ctypes.data_as(C.POINTER(C.c_uint8))
        self.L.orc_set(self.h, conv(x, (n, 3)), conv(v, (n, 3)), conv(F, (n, 9)), dg, conv(D, (n,)))

    def codes(self):
        """Ternary codes c_p = sum_k d_k 3^k (Eq. 7) as uint64."""
        dig = self.get()["digits"].astype(np.uint64)
        w = np.array([3 ** k for k in range(self.K)], dtype=np.uint64)
        return (dig * w).sum(axis=1) if self.K else np.zeros(self.n, np.uint64)

    def candidates(self):
        c = np.zeros(self.n, np.uint8)
        self.L.orc_candidates(self.h, c.ctypes.data_as(C.POINTER(C.c_uint8)))
        return c.astype(bool)

    def last_pairs(self):
        return self.L.orc_last_pairs(self.h)

    def grid_dump(self):
        cap = 27 * self.n + 8
        node = np.empty(cap, np.int64)
        code = np.empty(cap, np.uint64)
        m = np.empty(cap)
        vn = np.empty((cap, 3))
        vn1 = np.empty((cap, 3))
        vt = np.empty((cap, 3))
        k = self.L.orc_grid_dump(self.h, cap, node.ctypes.data_as(C.POINTER(C.c_int64)),
                                code.ctypes.data_as(C.POINTER(C.c_uint64)), _dp(m), _dp(vn), _dp(vn1), _dp(vt))
        return {"node": node[:k], "code": code[:k], "m": m[:k], "vn": vn[:k], "vn1": vn1[:k], "vt": vt[:k]}


def set_threads(n):
    """Threads of the oracle's loops with independent iterations (results do not
    depend on it)."""
    lib().orc_set_threads(int(n))


def get_threads():
    return lib().orc_get_threads()


# --- primitives, for the pins -------------------------------------------------

def shape(params, X):
    """(node[k], w[k], grad[k,3]) of the stencil at reference point X: k = 8 for the
    trilinear hat, 27 for the quadratic B-spline (params stencil = 1)."""
    P = make_params(params) if isinstance(params, dict) else params
    X = _f64(X, (3,))
    k = 27 if P.stencil == 1 else 8
    node = (C.c_long * 27)()
    w = np.empty(27)
    g = np.empty((27, 3))
    if lib().orc_shape(C.byref(P), _dp(X), node, _dp(w), _dp(g)):
        raise ValueError("outside grid")
    return np.array(list(node))[:k], w[:k].copy(), g[:k].copy()


def neo_hookean_P(E, nu, F):
    F = _f64(F, (9,))
    P = np.empty(9)
    lib().orc_neo_hookean_P(float(E), float(nu), _dp(F), _dp(P))
    return P.reshape(3, 3)


def neo_hookean_psi(E, nu, F):
    F = _f64(F, (9,))
    return lib().orc_neo_hookean_psi(float(E), float(nu), _dp(F))


def fcr_P(E, nu, F):
    F = _f64(F, (9,))
    P = np.empty(9)
    lib().orc_fcr_P(float(E), float(nu), _dp(F), _dp(P))
    return P.reshape(3, 3)


def fcr_psi(E, nu, F):
    F = _f64(F, (9,))
    return lib().orc_fcr_psi(float(E), float(nu), _dp(F))


def polar(F):
    F = _f64(F, (9,))
    R, S = np.empty(9), np.empty(9)
    if lib().orc_polar(_dp(F), _dp(R), _dp(S)):
        raise ValueError("det F <= 0")
    return R.reshape(3, 3), S.reshape(3, 3)


def vm_project(E, nu, sigma_y, Fe):
    """(projected F_e, yielded) of the von Mises projection."""
    Fe = _f64(Fe, (9,))
    out = np.empty(9)
    r = lib().orc_vm_project(float(E), float(nu), float(sigma_y), _dp(Fe), _dp(out))
    if r < 0:
        raise ValueError("det F_e <= 0")
    return out.reshape(3, 3), bool(r)


def visc_P(eta, F, Fdot):
    F, Fd = _f64(F, (9,)), _f64(Fdot, (9,))
    P = np.empty(9)
    lib().orc_visc_P(float(eta), _dp(F), _dp(Fd), _dp(P))
    return P.reshape(3, 3)


def conflict(a, b, K):
    return bool(lib().orc_conflict(int(a), int(b), int(K)))


def encode(digits):
    d = np.ascontiguousarray(np.asarray(digits, np.uint8))
    return int(lib().orc_encode(d.ctypes.data_as(C.POINTER(C.c_uint8)), len(d)))


def digit(code, k):
    return lib().orc_digit(int(code), int(k))


def couple(m, codes, K, f):
    """Eq. 8 at one node: m [S], codes [S], f [S,3] -> f_bar [S,3]."""
    m = _f64(m)
    S = len(m)
    f = _f64(f, (S, 3))
    c = np.ascontiguousarray(np.asarray(codes, np.uint64))
    out = np.empty((S, 3))
    lib().orc_couple(S, _dp(m), c.ctypes.data_as(C.POINTER(C.c_uint64)), int(K), _dp(f), _dp(out))
    return out


def label_digit(x, v, blade, dt, digit_now=0):
    x = _f64(x, (3,))
    v = _f64(v, (3,))
    B = make_blade(blade)
    return lib().orc_label_digit(_dp(x), _dp(v), C.byref(B), float(dt), int(digit_now))


def labels_on(X, u, v, digits, blades, dt):
    """Shared-input label pass: evaluates the band of every blade on FP32 state
    widened to FP64 (x = X + u, exact) and returns updated digits [n, K]."""
    X = np.asarray(X, np.float32).astype(np.float64)
    u = np.asarray(u, np.float32).astype(np.float64)
    x = np.ascontiguousarray(X + u)
    v = np.ascontiguousarray(np.asarray(v, np.float32).astype(np.float64))
    dig = np.array(digits, np.uint8, copy=True, order="C")
    n, K = dig.shape
    arr = (Blade * max(1, len(blades)))(*[make_blade(b) for b in blades])
    r = lib().orc_label_pass(n, _dp(x), _dp(v), dig.ctypes.data_as(C.POINTER(C.c_uint8)), K, arr,
                             len(blades), float(dt))
    if r < 0:
        raise ValueError("bad cut index")
    return dig
