"""Python binding of libtlmpm.so (argument marshalling only).

Every step of the method runs in the HIP kernels behind the C ABI of
include/tlmpm.h.  PyTorch provides the device workspace and the stream.  The
library must be built (``python -m paper_2609_27342_amd.build``); importing this
module on a machine without it raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtlmpm.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_SLOT_OVERFLOW, E_NONFINITE = range(6)
TOOL_LABELS, TOOL_CONTACT, TOOL_CUTTING, TOOL_ADVANCE = 1, 2, 4, 8
FIELD_X, FIELD_U, FIELD_V, FIELD_F, FIELD_CODE, FIELD_D, FIELD_DIGITS, FIELD_H = 1, 2, 4, 8, 16, 32, 64, 128
MAX_TOOLS = 4


class SceneDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("X", C.c_void_p), ("v0", C.c_void_p), ("vol0", C.c_void_p),
        ("mass", C.c_void_p), ("E", C.c_void_p),
        ("vol0_uniform", C.c_float), ("mass_uniform", C.c_float), ("E_uniform", C.c_float),
        ("nu", C.c_float), ("dx", C.c_double), ("origin", C.c_double * 3), ("cells", C.c_int32 * 3),
        ("dt", C.c_double), ("gravity", C.c_float * 3), ("flip_beta", C.c_float),
        ("s_R", C.c_float), ("s_n", C.c_float), ("gamma_k", C.c_float), ("gamma_c", C.c_float),
        ("mu_s", C.c_float), ("mu_d", C.c_float),
        ("material_contact", C.c_int32), ("floor_on", C.c_int32), ("floor_z", C.c_float),
        ("G_c", C.c_float), ("zeta", C.c_float), ("u_min", C.c_float),
        ("max_cuts", C.c_int32), ("single_field", C.c_int32), ("slot_capacity", C.c_int32),
        ("material", C.c_int32), ("viscosity", C.c_float), ("yield_stress", C.c_float),
        ("stencil", C.c_int32),
    ]


class Blade(C.Structure):
    _fields_ = [
        ("cut_index", C.c_int32), ("new_cut", C.c_int32),
        ("x_e", C.c_double * 3), ("n", C.c_double * 3), ("e", C.c_double * 3), ("d", C.c_double * 3),
        ("v_e", C.c_double * 3), ("half_len", C.c_double), ("half_width", C.c_double),
        ("b_back", C.c_double), ("b_lead", C.c_double),
    ]


class Tool(C.Structure):
    _fields_ = [
        ("blade", Blade), ("x_B", C.c_double * 3), ("v_B", C.c_double * 3), ("omega_B", C.c_double * 3),
        ("w_B", C.c_double), ("flags", C.c_uint32), ("reserved", C.c_int32),
        ("inv_mass", C.c_double), ("inv_inertia", C.c_double * 9),
    ]


_lib = None


class Tuning(C.Structure):
    _fields_ = [("pair_div", C.c_int32), ("pair_cap", C.c_int32), ("split_lo", C.c_int32), ("split_hi", C.c_int32),
                ("split_div", C.c_int32), ("split_cap", C.c_int32), ("one_stream_bricks", C.c_int32),
                ("pair_skip", C.c_int32)]


TUNING_KEYS = tuple(k for k, _ in Tuning._fields_)


class RigidBodyC(C.Structure):
    _fields_ = [
        ("x", C.c_double * 3), ("q", C.c_double * 4), ("v", C.c_double * 3), ("omega", C.c_double * 3),
        ("mass", C.c_double), ("inertia", C.c_double * 3),
    ]


def lib():
    """Load libtlmpm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtlmpm.so is not built; run python -m paper_2609_27342_amd.build")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.tlmpm_scene_footprint.argtypes = [C.POINTER(SceneDesc), C.POINTER(C.c_size_t)]
        L.tlmpm_create_scene.argtypes = [C.POINTER(SceneDesc), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.tlmpm_destroy_scene.argtypes = [vp]
        L.tlmpm_assign_labels.argtypes = [vp, C.POINTER(Blade), C.c_int32]
        L.tlmpm_step.argtypes = [vp, C.POINTER(Tool), C.c_int32, C.c_int32, C.POINTER(C.c_double)]
        L.tlmpm_read_state.argtypes = [vp, C.c_uint32, C.POINTER(vp)]
        L.tlmpm_write_state.argtypes = [vp, C.c_uint32, C.POINTER(vp)]
        L.tlmpm_get_status.argtypes = [vp, C.POINTER(C.c_int32)]
        L.tlmpm_slot_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        L.tlmpm_contact_stats.argtypes = [vp, C.POINTER(C.c_double)]
        L.tlmpm_slot_histogram.argtypes = [vp, C.POINTER(C.c_int64)]
        dp = C.POINTER(C.c_double)
        L.tlmpm_rigid_step.argtypes = [C.POINTER(RigidBodyC), dp, dp, C.c_double]
        L.tlmpm_rigid_tool.argtypes = [C.POINTER(RigidBodyC), C.POINTER(Blade), C.c_uint32, C.POINTER(Tool)]
        L.tlmpm_profile_enable.argtypes = [vp, C.c_int32]
        L.tlmpm_profile_read.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.tlmpm_batch_footprint.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(C.c_size_t)]
        L.tlmpm_batch_scene_bytes.argtypes = [C.POINTER(SceneDesc), C.POINTER(C.c_size_t)]
        L.tlmpm_surface_footprint.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.tlmpm_surface_build.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]
        L.tlmpm_surface_read.argtypes = [vp, vp, C.c_size_t, vp, vp, vp, vp, vp]
        L.tlmpm_batch_create.argtypes = [C.POINTER(vp), C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.tlmpm_batch_create_static.argtypes = [C.POINTER(vp), C.c_int32, vp, C.POINTER(vp)]
        L.tlmpm_batch_destroy.argtypes = [vp]
        L.tlmpm_batch_step.argtypes = [vp, C.POINTER(Tool), C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_double)]
        L.tlmpm_batch_sync.argtypes = [vp]
        L.tlmpm_batch_profile_enable.argtypes = [vp, C.c_int32]
        L.tlmpm_set_graphs.argtypes = [vp, C.c_int32]
        L.tlmpm_batch_set_graphs.argtypes = [vp, C.c_int32]
        L.tlmpm_batch_profile_read.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.tlmpm_set_tuning.argtypes = [C.POINTER(Tuning)]
        L.tlmpm_get_tuning.argtypes = [C.POINTER(Tuning)]
        L.tlmpm_last_error.restype = C.c_char_p
        for f in ("tlmpm_scene_footprint", "tlmpm_create_scene", "tlmpm_destroy_scene", "tlmpm_assign_labels",
                  "tlmpm_step", "tlmpm_read_state", "tlmpm_write_state", "tlmpm_get_status", "tlmpm_slot_stats", "tlmpm_slot_histogram", "tlmpm_contact_stats", "tlmpm_rigid_step", "tlmpm_rigid_tool",
                  "tlmpm_profile_enable", "tlmpm_profile_read", "tlmpm_batch_footprint", "tlmpm_batch_scene_bytes",
                  "tlmpm_surface_footprint", "tlmpm_surface_build", "tlmpm_surface_read",
                  "tlmpm_batch_create", "tlmpm_batch_create_static",
                  "tlmpm_batch_destroy", "tlmpm_batch_step", "tlmpm_batch_sync", "tlmpm_batch_profile_enable",
                  "tlmpm_batch_profile_read", "tlmpm_set_graphs", "tlmpm_batch_set_graphs", "tlmpm_set_tuning",
                  "tlmpm_get_tuning"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def get_tuning():
    """The launch-shape settings new scenes take (tlmpm_get_tuning), as a dict."""
    t = Tuning()
    _check(lib().tlmpm_get_tuning(C.byref(t)))
    return {k: int(getattr(t, k)) for k in TUNING_KEYS}


def set_tuning(tuning=None, **kw):
    """Sets the launch-shape settings of scenes created from now on
    (tlmpm_set_tuning): keys of TUNING_KEYS, unnamed ones unchanged; set_tuning(None)
    with no keywords restores the defaults."""
    if tuning is None and not kw:
        _check(lib().tlmpm_set_tuning(None))
        return
    cur = get_tuning()
    cur.update(tuning or {})
    cur.update(kw)
    unknown = set(cur) - set(TUNING_KEYS)
    if unknown:
        raise ValueError(f"unknown tuning keys {sorted(unknown)}")
    t = Tuning(**{k: int(cur[k]) for k in TUNING_KEYS})
    _check(lib().tlmpm_set_tuning(C.byref(t)))


class TlmpmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tlmpm status {code}: {msg}")
        self.code = code


def _check(code):
    if code != OK:
        raise TlmpmError(code, lib().tlmpm_last_error().decode())


def _vec(dst, src):
    src = np.asarray(src, np.float64)
    for i in range(3):
        dst[i] = float(src[i])


def make_blade(b):
    B = Blade()
    B.cut_index = int(b["cut_index"])
    B.new_cut = int(b.get("new_cut", 0))
    for k in ("x_e", "n", "e", "d", "v_e"):
        _vec(getattr(B, k), b[k])
    for k in ("half_len", "half_width", "b_back", "b_lead"):
        setattr(B, k, float(b[k]))
    return B


def make_tool(t):
    T = Tool()
    T.blade = make_blade(t["blade"])
    for k in ("x_B", "v_B", "omega_B"):
        _vec(getattr(T, k), t.get(k, (0.0, 0.0, 0.0)))
    T.w_B = float(t.get("w_B", 0.0))
    T.inv_mass = float(t.get("inv_mass", 0.0))
    ii = np.asarray(t.get("inv_inertia", np.zeros(9)), dtype=np.float64).reshape(9)
    for i in range(9):
        T.inv_inertia[i] = float(ii[i])
    fl = 0
    if t.get("labels"):
        fl |= TOOL_LABELS
    if t.get("contact"):
        fl |= TOOL_CONTACT
    if t.get("cutting"):
        fl |= TOOL_CUTTING
    if t.get("advance"):
        fl |= TOOL_ADVANCE
    T.flags = fl
    return T


def tool_dict(T):
    """Tool dict (the form Scene.step and Batch.step take) of a Tool structure."""
    b = T.blade
    blade = dict(cut_index=b.cut_index, new_cut=b.new_cut, half_len=b.half_len, half_width=b.half_width,
                 b_back=b.b_back, b_lead=b.b_lead)
    for k in ("x_e", "n", "e", "d", "v_e"):
        blade[k] = np.array(getattr(b, k)[:], dtype=np.float64)
    return dict(blade=blade, x_B=np.array(T.x_B[:]), v_B=np.array(T.v_B[:]), omega_B=np.array(T.omega_B[:]),
                w_B=T.w_B, inv_mass=T.inv_mass, inv_inertia=np.array(T.inv_inertia[:]),
                labels=bool(T.flags & TOOL_LABELS), contact=bool(T.flags & TOOL_CONTACT),
                cutting=bool(T.flags & TOOL_CUTTING), advance=bool(T.flags & TOOL_ADVANCE))


class RigidBody:
    """A free rigid tool body (tlmpm_rigid_body): x (centre of mass), q (w, x, y, z),
    v, omega (world), mass, principal inertia (body axes)."""

    def __init__(self, x, q, v, omega, mass, inertia):
        self.c = RigidBodyC()
        _vec(self.c.x, x)
        for i in range(4):
            self.c.q[i] = float(q[i])
        _vec(self.c.v, v)
        _vec(self.c.omega, omega)
        self.c.mass = float(mass)
        _vec(self.c.inertia, inertia)

    def step(self, wrench, gravity, h):
        """tlmpm_rigid_step: advance by h under wrench (force, torque) and gravity."""
        w = (C.c_double * 6)(*[float(a) for a in np.asarray(wrench, np.float64).reshape(6)])
        g = (C.c_double * 3)(*[float(a) for a in np.asarray(gravity, np.float64).reshape(3)])
        _check(lib().tlmpm_rigid_step(C.byref(self.c), w, g, float(h)))

    def tool(self, blade_body, labels=True, contact=True, cutting=True):
        """tlmpm_rigid_tool: the tool dict of a blade fixed to the body (blade_body in
        body axes relative to the centre of mass)."""
        B = make_blade(dict(blade_body, v_e=(0.0, 0.0, 0.0)))
        fl = (TOOL_LABELS if labels else 0) | (TOOL_CONTACT if contact else 0) | (TOOL_CUTTING if cutting else 0)
        T = Tool()
        _check(lib().tlmpm_rigid_tool(C.byref(self.c), C.byref(B), fl, C.byref(T)))
        return tool_dict(T)

    def state(self):
        return dict(x=np.array(self.c.x[:]), q=np.array(self.c.q[:]), v=np.array(self.c.v[:]),
                    omega=np.array(self.c.omega[:]))


def make_desc(scene, keep):
    """SceneDesc from a workload scene dict; arrays kept alive in `keep`."""
    p = scene["params"]
    d = SceneDesc()
    X = np.ascontiguousarray(scene["X"], np.float32)
    keep.append(X)
    d.n = X.shape[0]
    d.X = X.ctypes.data
    if scene.get("v0") is not None:
        v0 = np.ascontiguousarray(scene["v0"], np.float32)
        keep.append(v0)
        d.v0 = v0.ctypes.data
    for name, arr_key in (("vol0", "vol0"), ("mass", "mass"), ("E", "E")):
        a = np.asarray(scene[arr_key], np.float32)
        if a.size == 0:  # no particles: any positive uniform value
            setattr(d, name + "_uniform" if name != "E" else "E_uniform", 1.0)
        elif a.ndim == 0 or np.all(a == a.flat[0]):
            setattr(d, name + "_uniform" if name != "E" else "E_uniform", float(a.flat[0]))
        else:
            a = np.ascontiguousarray(a)
            keep.append(a)
            setattr(d, name, a.ctypes.data)
    d.nu = float(p["nu"])
    d.dx = float(p["dx"])
    _vec(d.origin, p["origin"])
    for i in range(3):
        d.cells[i] = int(p["cells"][i])
    d.dt = float(p["dt"])
    g = p.get("gravity", (0.0, 0.0, -9.81))
    for i in range(3):
        d.gravity[i] = float(g[i])
    d.flip_beta = float(p.get("flip_beta", 0.95))
    for k in ("s_R", "s_n", "gamma_k", "gamma_c", "mu_s", "mu_d", "floor_z", "G_c", "zeta", "u_min"):
        setattr(d, k, float(p[k]))
    d.material_contact = int(p.get("material_contact", 0))
    d.floor_on = int(p.get("floor_on", 0))
    d.max_cuts = int(p.get("max_cuts", 4))
    d.single_field = int(p.get("single_field", 0))
    d.slot_capacity = int(p.get("slot_capacity", 0))
    d.material = int(p.get("material", 0))
    d.viscosity = float(p.get("viscosity", 0.0))
    d.yield_stress = float(p.get("yield_stress", 0.0))
    d.stencil = int(p.get("stencil", 0))
    return d


def footprint(scene):
    keep = []
    d = make_desc(scene, keep)
    nb = C.c_size_t()
    _check(lib().tlmpm_scene_footprint(C.byref(d), C.byref(nb)))
    return nb.value


def batch_scene_bytes(scene):
    """Bound on the bytes the scene adds to a batch workspace (tlmpm_batch_scene_bytes)."""
    keep = []
    d = make_desc(scene, keep)
    nb = C.c_size_t()
    _check(lib().tlmpm_batch_scene_bytes(C.byref(d), C.byref(nb)))
    return nb.value


class Scene:
    """A scene resident on the current torch device.  `stream` is a torch stream
    (default: the current one)."""

    def __init__(self, scene, stream=None, workspace=None):
        import torch
        L = lib()
        self._keep = []
        self.desc = make_desc(scene, self._keep)
        self.n = int(self.desc.n)
        self.max_cuts = int(self.desc.max_cuts)
        nb = C.c_size_t()
        _check(L.tlmpm_scene_footprint(C.byref(self.desc), C.byref(nb)))
        self.bytes = nb.value
        if workspace is None:
            workspace = torch.empty(self.bytes, dtype=torch.uint8, device="cuda")
        assert workspace.numel() >= self.bytes and workspace.is_cuda
        self.ws = workspace
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(L.tlmpm_create_scene(C.byref(self.desc), C.c_void_p(workspace.data_ptr()), self.bytes,
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _check(lib().tlmpm_destroy_scene(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def assign_labels(self, blades):
        arr = (Blade * max(1, len(blades)))(*[make_blade(b) for b in blades])
        _check(lib().tlmpm_assign_labels(self.h, arr, len(blades)))

    def step(self, tools=(), n_substeps=1, wrench=False):
        nt = len(tools)
        arr = (Tool * max(1, nt))(*[make_tool(t) for t in tools])
        w = np.zeros((max(1, nt), 6))
        wp = w.ctypes.data_as(C.POINTER(C.c_double)) if wrench else None
        _check(lib().tlmpm_step(self.h, arr, nt, int(n_substeps), wp))
        return w[:nt] if wrench else None

    def read(self, fields=("u", "v", "F", "code", "D", "digits")):
        n, K = self.n, self.max_cuts
        spec = {"X": (FIELD_X, (n, 3), np.float32), "u": (FIELD_U, (n, 3), np.float32),
                "v": (FIELD_V, (n, 3), np.float32), "F": (FIELD_F, (n, 3, 3), np.float32),
                "code": (FIELD_CODE, (n,), np.uint64), "D": (FIELD_D, (n,), np.float32),
                "digits": (FIELD_DIGITS, (n, K), np.uint8), "H": (FIELD_H, (n, 3, 3), np.float32)}
        order = sorted(fields, key=lambda f: spec[f][0])
        mask = 0
        outs = {}
        for f in order:
            bit, shape, dt = spec[f]
            mask |= bit
            outs[f] = np.zeros(shape, dt)
        ptrs = (C.c_void_p * max(1, len(order)))(*[outs[f].ctypes.data for f in order])
        _check(lib().tlmpm_read_state(self.h, mask, ptrs))
        return outs

    def write(self, **fields):
        spec = {"u": (FIELD_U, np.float32), "v": (FIELD_V, np.float32), "F": (FIELD_F, np.float32),
                "D": (FIELD_D, np.float32), "digits": (FIELD_DIGITS, np.uint8), "H": (FIELD_H, np.float32)}
        order = sorted(fields, key=lambda f: spec[f][0])
        mask = 0
        keep = []
        for f in order:
            bit, dt = spec[f]
            mask |= bit
            keep.append(np.ascontiguousarray(fields[f], dt))
        ptrs = (C.c_void_p * max(1, len(order)))(*[a.ctypes.data for a in keep])
        _check(lib().tlmpm_write_state(self.h, mask, ptrs))

    def status(self):
        st = C.c_int32()
        _check(lib().tlmpm_get_status(self.h, C.byref(st)))
        return st.value

    def status_detail(self):
        """(status, the device status bits as text, empty when OK)."""
        st = self.status()
        return st, (lib().tlmpm_last_error().decode() if st else "")

    KERNEL_CLASSES = ("p2g", "g2p", "labels", "slots", "contact", "other")

    def graphs(self, enable=True):
        """Replay pairs of substeps as captured HIP graphs (bitwise the same results)."""
        _check(lib().tlmpm_set_graphs(self.h, int(bool(enable))))

    def profile(self, enable=True):
        """enable: True / 1 every launch timed (each kernel alone, one stream);
        "transfers" / 2 only P2G and G2P, the launch arrangement unchanged; False off."""
        mode = 2 if enable == "transfers" else int(enable)
        _check(lib().tlmpm_profile_enable(self.h, mode))

    def profile_read(self):
        """{class: (total ms, launches)} since the last read (synchronises)."""
        ms = (C.c_double * 6)()
        cnt = (C.c_int64 * 6)()
        _check(lib().tlmpm_profile_read(self.h, 6, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KERNEL_CLASSES)}

    def surface(self):
        """The surface of the current side codes (tlmpm_surface_*): dict of x [nv,3]
        current and X [nv,3] reference vertex positions, code [nv], quads [nq,4] and
        cut [nq] (bool)."""
        import torch
        L = lib()
        nb = C.c_size_t()
        _check(L.tlmpm_surface_footprint(self.h, C.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        counts = (C.c_int64 * 2)()
        need = C.c_size_t()
        r = L.tlmpm_surface_build(self.h, C.c_void_p(ws.data_ptr()), nb.value, counts, C.byref(need))
        if r == E_NOMEM and need.value > nb.value:
            ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
            r = L.tlmpm_surface_build(self.h, C.c_void_p(ws.data_ptr()), need.value, counts, C.byref(need))
        _check(r)
        nv, nq = counts[0], counts[1]
        out = {"x": np.zeros((nv, 3), np.float32), "X": np.zeros((nv, 3), np.float32),
               "code": np.zeros(nv, np.uint64), "quads": np.zeros((nq, 4), np.int32), "cut": np.zeros(nq, np.uint8)}
        _check(L.tlmpm_surface_read(self.h, C.c_void_p(ws.data_ptr()), ws.numel(), out["x"].ctypes.data,
                                    out["X"].ctypes.data, out["code"].ctypes.data, out["quads"].ctypes.data,
                                    out["cut"].ctypes.data))
        out["cut"] = out["cut"].astype(bool)
        return out

    def slot_stats(self):
        tot = C.c_int64()
        mx = C.c_int32()
        _check(lib().tlmpm_slot_stats(self.h, C.byref(tot), C.byref(mx)))
        return tot.value, mx.value

    def slot_histogram(self):
        """Nodes by number of logical-grid slots: list h, h[c] nodes with c slots."""
        h = (C.c_int64 * 17)()
        _check(lib().tlmpm_slot_histogram(self.h, h))
        return [int(x) for x in h]

    def contact_stats(self):
        """Material-contact search of the last substep: candidates, buckets,
        occupied buckets, buckets beyond their inline records, largest bucket
        count, bin edge (m), pairs in contact, candidates whose search was skipped
        (no partner possible)."""
        out = (C.c_double * 8)()
        _check(lib().tlmpm_contact_stats(self.h, out))
        keys = ("candidates", "buckets", "occupied", "overflowing", "max_count", "bin_edge", "pairs", "skipped")
        return {k: (out[i] if k == "bin_edge" else int(out[i])) for i, k in enumerate(keys)}


class Batch:
    """Scenes advanced together by shared kernel launches.  While the batch is
    open its scenes refuse single-scene calls; close() releases them."""

    def __init__(self, scenes, stream=None, workspace=None, static=False):
        """static=True: the workspace is the library's per-device static array
        (tlmpm_batch_create_static), nothing is allocated."""
        import torch
        L = lib()
        self.scenes = list(scenes)
        n = len(self.scenes)
        self._hs = (C.c_void_p * max(1, n))(*[s.h for s in self.scenes])
        nb = C.c_size_t()
        _check(L.tlmpm_batch_footprint(self._hs, n, C.byref(nb)))
        self.bytes = nb.value
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        if static:
            assert workspace is None
            self.ws = None
            _check(L.tlmpm_batch_create_static(self._hs, n, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        else:
            if workspace is None:
                workspace = torch.empty(self.bytes, dtype=torch.uint8, device="cuda")
            assert workspace.numel() >= self.bytes and workspace.is_cuda
            self.ws = workspace
            _check(L.tlmpm_batch_create(self._hs, n, C.c_void_p(workspace.data_ptr()), self.bytes,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self._tools = (Tool * (MAX_TOOLS * max(1, n)))()
        self._counts = (C.c_int32 * max(1, n))()

    def close(self):
        if getattr(self, "h", None):
            _check(lib().tlmpm_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def step(self, tools_per_scene, n_substeps=1, wrench=False):
        """tools_per_scene: one list of tool dicts per scene.  Returns, with
        wrench=True, an array [n_scenes][4][6] of interval-averaged wrenches."""
        n = len(self.scenes)
        assert len(tools_per_scene) == n
        for s, tl in enumerate(tools_per_scene):
            assert len(tl) <= MAX_TOOLS
            self._counts[s] = len(tl)
            for t, tool in enumerate(tl):
                self._tools[s * MAX_TOOLS + t] = make_tool(tool)
        w = np.zeros((max(1, n), MAX_TOOLS, 6))
        wp = w.ctypes.data_as(C.POINTER(C.c_double)) if wrench else None
        _check(lib().tlmpm_batch_step(self.h, self._tools, self._counts, int(n_substeps), wp))
        return w[:n] if wrench else None

    def sync(self):
        _check(lib().tlmpm_batch_sync(self.h))

    def graphs(self, enable=True):
        _check(lib().tlmpm_batch_set_graphs(self.h, int(bool(enable))))

    def profile(self, enable=True):
        """As Scene.profile."""
        mode = 2 if enable == "transfers" else int(enable)
        _check(lib().tlmpm_batch_profile_enable(self.h, mode))

    def profile_read(self):
        """{class: (total ms, launches)} since the last read (synchronises)."""
        ms = (C.c_double * 6)()
        cnt = (C.c_int64 * 6)()
        _check(lib().tlmpm_batch_profile_read(self.h, 6, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(Scene.KERNEL_CLASSES)}
