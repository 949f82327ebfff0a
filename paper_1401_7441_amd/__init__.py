"""MI355X-native local-Hamiltonian path of linear-scaling Daubechies-wavelet
DFT (Mohr et al., arXiv:1401.7441), Python binding.

The compute lives in libwvl.so (HIP kernels for gfx950 behind the C ABI of
include/wvl.h).  This module only marshals arguments: numpy arrays for the
host-side descriptions (localization regions, segment lists), torch tensors
for device buffers and streams.  Every operation runs in the library's
kernels; there is no fallback, and importing the package fails if the
library has not been built (``python -m paper_1401_7441_amd.build``).

Names follow the C ABI: build_locregs, Context (wvl_create), Plan
(wvl_plan_create), uncompress, compress, apply_local_ham, kinetic,
sparse_overlap.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch first: its HIP runtime must be the one libwvl.so binds to (the library
# needs libamdhip64.so.7, which the already-loaded torch runtime satisfies);
# torch's streams and device pointers are only meaningful to that runtime.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwvl.so")

WVL_OK, WVL_EINVAL, WVL_ENOMEM, WVL_EDEVICE, WVL_EUNSUPPORTED = 0, -1, -2, -3, -4
F32, F64 = 0, 1
KIN, POT = 1, 2

SEG_DTYPE = np.dtype([("i1s", "<i4"), ("i1e", "<i4"), ("i2", "<i4"), ("i3", "<i4"),
                      ("off", "<i8")], align=True)
LOCREG_DTYPE = np.dtype([
    ("center", "<f8", (3,)), ("radius", "<f8"), ("fine_radius", "<f8"),
    ("ext", "<i4"), ("lo", "<i4", (3,)), ("dims", "<i4", (3,)), ("pad_", "<i4"),
    ("seg_c", "<i8"), ("nseg_c", "<i8"), ("seg_f", "<i8"), ("nseg_f", "<i8"),
    ("oseg_c", "<i8"), ("noseg_c", "<i8"), ("oseg_f", "<i8"), ("noseg_f", "<i8"),
    ("coef_off", "<i8"), ("n_c", "<i8"), ("n_f", "<i8"),
    ("ocoef_off", "<i8"), ("on_c", "<i8"), ("on_f", "<i8")], align=True)

EXPORTED = ("wvl_build_locregs", "wvl_create", "wvl_destroy", "wvl_last_error",
            "wvl_plan_create", "wvl_plan_destroy", "wvl_plan_info_get", "wvl_uncompress",
            "wvl_compress", "wvl_apply_local_ham", "wvl_apply_local_ham_conf",
            "wvl_apply_local_ham_static", "wvl_kinetic",
            "wvl_sparse_overlap", "wvl_synthesize", "wvl_density", "wvl_foe", "wvl_gradient",
            "wvl_update", "wvl_precondition", "wvl_graph_create", "wvl_graph_launch",
            "wvl_graph_destroy",
            "wvl_plan_autotune", "wvl_plan_set_schedule",
            "wvl_profile_enable", "wvl_profile_reset", "wvl_profile_count", "wvl_profile_read")


class WvlError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"wvl status {status}: {msg}")
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("n", ctypes.c_int32 * 3)]


class _TunePoint(ctypes.Structure):
    _fields_ = [("nbins", ctypes.c_int32), ("kin_mfma", ctypes.c_int32), ("ms", ctypes.c_double)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("nsf", "in_coefs", "out_coefs", "in_box", "out_box",
                                               "workspace_f32", "workspace_f64", "chunks",
                                               "fine_box")]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1401_7441_amd.build` (no fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    runtimes.add(line.split()[-1])
    except OSError:
        pass
    if len(runtimes) > 1:
        raise ImportError(f"two HIP runtimes are loaded in this process ({sorted(runtimes)}); "
                          "import torch before loading libwvl.so")
    P, I32, I64, U32, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                           ctypes.c_double)
    sig = {
        "wvl_build_locregs": [ctypes.POINTER(_Grid), I32, P, P, P, I32, P, P,
                              ctypes.POINTER(I64)],
        "wvl_create": [ctypes.POINTER(P), ctypes.POINTER(_Grid), P],
        "wvl_destroy": [P],
        "wvl_last_error": [P],
        "wvl_plan_create": [P, I32, P, P, I64, ctypes.c_size_t, ctypes.POINTER(P),
                            ctypes.POINTER(ctypes.c_size_t)],
        "wvl_plan_destroy": [P],
        "wvl_plan_info_get": [P, ctypes.POINTER(_PlanInfo)],
        "wvl_uncompress": [P, ctypes.c_int, P, P],
        "wvl_compress": [P, ctypes.c_int, P, P],
        "wvl_apply_local_ham": [P, ctypes.c_int, U32, P, P, P, P, P, P],
        "wvl_kinetic": [P, ctypes.c_int, P, P, P, P],
        "wvl_apply_local_ham_conf": [P, ctypes.c_int, U32, P, P, P, P, P, P, P],
        "wvl_apply_local_ham_static": [P, ctypes.c_int, U32, P, P, P, P, P],
        "wvl_sparse_overlap": [P, P, ctypes.c_int, P, ctypes.c_int, ctypes.POINTER(I64), P, P, P],
        "wvl_synthesize": [P, ctypes.c_int, P, P, P],
        "wvl_foe": [P, P, P, I32, D, D, D, D, P, ctypes.POINTER(D), ctypes.POINTER(D), P,
                    ctypes.c_size_t],
        "wvl_density": [P, ctypes.c_int, P, P, P, P, I64, P, P],
        "wvl_gradient": [P, ctypes.c_int, P, P, P, P, P, P, P, ctypes.c_size_t],
        "wvl_update": [P, ctypes.c_int, D, P, P, P],
        "wvl_precondition": [P, ctypes.c_int, P, P, P, I32, P, P, P],
        "wvl_graph_create": [P, ctypes.c_int, U32, P, P, P, P, P, P, P, P, ctypes.POINTER(P)],
        "wvl_graph_launch": [P],
        "wvl_graph_destroy": [P],
        "wvl_plan_autotune": [P, ctypes.c_int, U32, P, P, P, P, I32, ctypes.POINTER(_TunePoint),
                              I32, ctypes.POINTER(I32), ctypes.POINTER(_TunePoint)],
        "wvl_plan_set_schedule": [P, I32, I32],
        "wvl_profile_enable": [P, ctypes.c_int],
        "wvl_profile_reset": [P],
        "wvl_profile_count": [],
        "wvl_profile_read": [P, I32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(I64),
                             ctypes.POINTER(D)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.wvl_destroy.restype = None
    lib.wvl_plan_destroy.restype = None
    lib.wvl_graph_destroy.restype = None
    lib.wvl_last_error.restype = ctypes.c_char_p
    return lib


_lib = None
_load_error = None
try:
    _lib = _load()
except (OSError, AttributeError, ImportError) as _e:   # missing or stale build
    _load_error = _e


def lib():
    """The loaded libwvl.so.  Raises when it is missing or stale: there is no
    fallback implementation."""
    if _lib is None:
        raise ImportError(f"libwvl.so is not usable ({_load_error}); build it with "
                          "`python -m paper_1401_7441_amd.build`")
    return _lib


def _check(status, ctx=None):
    if status != WVL_OK:
        msg = lib().wvl_last_error(ctx)
        raise WvlError(status, msg.decode() if msg else "")


def _grid(h, n):
    g = _Grid()
    g.h = float(h)
    for a in range(3):
        g.n[a] = int(n[a])
    return g


def build_locregs(h, grid_n, centers, radii, fine_radii, ext):
    """wvl_build_locregs: sphere localization regions -> (locregs, segs) as
    numpy structured arrays (LOCREG_DTYPE, SEG_DTYPE)."""
    c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(radii, dtype=np.float64)
    f = np.ascontiguousarray(fine_radii, dtype=np.float64)
    nsf = len(c)
    g = _grid(h, grid_n)
    lr = np.zeros(nsf, LOCREG_DTYPE)
    # one call with a generous capacity (rows of the output boxes, several
    # runs per row); a second, exact one only when it was too small
    rows = (2.0 * (r + ext * float(h)) / float(h) + 3.0) ** 2
    cap = int(np.sum(6.0 * rows)) + 16
    segs = np.zeros(cap, SEG_DTYPE)
    n = ctypes.c_int64(cap)
    st = lib().wvl_build_locregs(ctypes.byref(g), nsf, c.ctypes.data, r.ctypes.data,
                                 f.ctypes.data, int(ext), lr.ctypes.data, segs.ctypes.data,
                                 ctypes.byref(n))
    if st != 0 and n.value > cap:
        segs = np.zeros(n.value, SEG_DTYPE)
        st = lib().wvl_build_locregs(ctypes.byref(g), nsf, c.ctypes.data, r.ctypes.data,
                                     f.ctypes.data, int(ext), lr.ctypes.data, segs.ctypes.data,
                                     ctypes.byref(n))
    _check(st)
    return lr, segs[:n.value].copy()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dtype_code(*tensors):
    import torch
    dts = {t.dtype for t in tensors if t is not None}
    if len(dts) != 1:
        raise WvlError(WVL_EINVAL, f"mixed or missing dtypes {dts}")
    dt = dts.pop()
    if dt == torch.float32:
        return F32
    if dt == torch.float64:
        return F64
    raise WvlError(WVL_EINVAL, f"unsupported dtype {dt}")


def _need_cuda(*tensors):
    for t in tensors:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise WvlError(WVL_EINVAL, "device buffers must be contiguous GPU tensors")


class Context:
    """wvl_create: a grid (spacing h, coarse points n) bound to a HIP stream
    (a torch.cuda.Stream; None = torch's current stream)."""

    def __init__(self, h, grid_n, stream=None):
        import torch
        self.h = float(h)
        self.grid_n = tuple(int(v) for v in grid_n)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._ptr = ctypes.c_void_p()
        g = _grid(h, grid_n)
        _check(lib().wvl_create(ctypes.byref(self._ptr), ctypes.byref(g),
                               ctypes.c_void_p(self.stream.cuda_stream)))

    @property
    def handle(self):
        return self._ptr

    def profile(self, enable=True):
        """Bracket every kernel launch with HIP events on this context's stream."""
        _check(lib().wvl_profile_enable(self._ptr, int(bool(enable))), self._ptr)

    def profile_reset(self):
        _check(lib().wvl_profile_reset(self._ptr), self._ptr)

    def profile_read(self):
        """{kernel kind: (launches, total_ms)} of the traced launches so far."""
        out = {}
        for k in range(lib().wvl_profile_count()):
            name = ctypes.c_char_p()
            n = ctypes.c_int64()
            ms = ctypes.c_double()
            _check(lib().wvl_profile_read(self._ptr, k, ctypes.byref(name), ctypes.byref(n),
                                         ctypes.byref(ms)), self._ptr)
            out[name.value.decode()] = (int(n.value), float(ms.value))
        return out

    def close(self):
        if self._ptr:
            lib().wvl_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """wvl_plan_create: validated, device-resident batch of localization
    regions.  `max_workspace` bounds the FP64 workspace in bytes (0: none)."""

    def __init__(self, ctx: Context, locregs, segs, max_workspace=0):
        self.ctx = ctx
        self.locregs = np.ascontiguousarray(locregs, dtype=LOCREG_DTYPE)
        self.segs = np.ascontiguousarray(segs, dtype=SEG_DTYPE)
        self._ptr = ctypes.c_void_p()
        ws = ctypes.c_size_t(0)
        _check(lib().wvl_plan_create(ctx.handle, len(self.locregs), self.locregs.ctypes.data,
                                    self.segs.ctypes.data, len(self.segs), int(max_workspace),
                                    ctypes.byref(self._ptr), ctypes.byref(ws)), ctx.handle)
        self.info = self._read_info()

    def _read_info(self):
        info = _PlanInfo()
        _check(lib().wvl_plan_info_get(self._ptr, ctypes.byref(info)), self.ctx.handle)
        return {k: int(getattr(info, k)) for k, _ in _PlanInfo._fields_}

    @property
    def nsf(self):
        return self.info["nsf"]

    def workspace_bytes(self, dtype_code):
        return self.info["workspace_f64" if dtype_code == F64 else "workspace_f32"]

    def new_workspace(self, dtype):
        """A uint8 device tensor large enough for `dtype` (torch.float32/64)."""
        import torch
        code = F64 if dtype == torch.float64 else F32
        return torch.empty(max(1, self.workspace_bytes(code)), dtype=torch.uint8, device="cuda")

    def close(self):
        if self._ptr:
            lib().wvl_plan_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_sizes(plan, psi_c, hpsi_c, e_kin, e_pot, workspace, dt):
    if psi_c.numel() < plan.info["in_coefs"]:
        raise WvlError(WVL_EINVAL, "input coefficient buffer smaller than the plan's layout")
    if hpsi_c.numel() < plan.info["out_coefs"]:
        raise WvlError(WVL_EINVAL, "output coefficient buffer smaller than the plan's layout")
    for e in (e_kin, e_pot):
        if e is not None and (e.dtype.itemsize != 8 or e.numel() < plan.nsf):
            raise WvlError(WVL_EINVAL, "energy buffers must be float64 with nsf entries")
    if workspace is not None and workspace.numel() * workspace.element_size() < \
            plan.workspace_bytes(dt):
        raise WvlError(WVL_EINVAL, "workspace smaller than the plan needs")


def uncompress(plan: Plan, psi_c, psi_box):
    _need_cuda(psi_c, psi_box)
    dt = _dtype_code(psi_c, psi_box)
    if psi_c.numel() < plan.info["in_coefs"] or psi_box.numel() < plan.info["in_box"]:
        raise WvlError(WVL_EINVAL, "buffer smaller than the plan's layout")
    _check(lib().wvl_uncompress(plan._ptr, dt, _ptr(psi_c), _ptr(psi_box)), plan.ctx.handle)


def compress(plan: Plan, box, hpsi_c):
    _need_cuda(box, hpsi_c)
    dt = _dtype_code(box, hpsi_c)
    if box.numel() < plan.info["out_box"] or hpsi_c.numel() < plan.info["out_coefs"]:
        raise WvlError(WVL_EINVAL, "buffer smaller than the plan's layout")
    _check(lib().wvl_compress(plan._ptr, dt, _ptr(box), _ptr(hpsi_c)), plan.ctx.handle)


def apply_local_ham(plan: Plan, psi_c, pot, hpsi_c, e_kin=None, e_pot=None, workspace=None,
                    terms=KIN | POT, conf=None):
    """wvl_apply_local_ham (wvl_apply_local_ham_conf when `conf`, a float64
    device tensor [nsf] of confinement prefactors, is given); e_kin / e_pot
    are float64 device tensors [nsf] or None."""
    _need_cuda(psi_c, pot, hpsi_c, e_kin, e_pot, workspace, conf)
    if conf is not None and (conf.dtype.itemsize != 8 or conf.numel() < plan.nsf):
        raise WvlError(WVL_EINVAL, "conf must be float64 with nsf entries")
    dt = _dtype_code(psi_c, pot, hpsi_c)
    _check_sizes(plan, psi_c, hpsi_c, e_kin, e_pot, workspace, dt)
    if pot is not None:
        n = plan.ctx.grid_n
        need = (2 * n[0] + 29) * (2 * n[1] + 29) * (2 * n[2] + 29)
        if pot.numel() != need:
            raise WvlError(WVL_EINVAL, f"potential has {pot.numel()} points, the grid needs {need}")
    if workspace is None:
        workspace = plan.new_workspace(psi_c.dtype)
    if conf is not None:
        _check(lib().wvl_apply_local_ham_conf(plan._ptr, dt, int(terms), _ptr(psi_c), _ptr(pot),
                                              _ptr(conf), _ptr(hpsi_c), _ptr(e_kin), _ptr(e_pot),
                                              _ptr(workspace)), plan.ctx.handle)
        return
    _check(lib().wvl_apply_local_ham(plan._ptr, dt, int(terms), _ptr(psi_c), _ptr(pot),
                                    _ptr(hpsi_c), _ptr(e_kin), _ptr(e_pot), _ptr(workspace)),
           plan.ctx.handle)


STATIC_WORKSPACE_BYTES = 128 << 20     # WVL_STATIC_WORKSPACE_BYTES


def apply_local_ham_static(plan: Plan, psi_c, pot, hpsi_c, e_kin=None, e_pot=None,
                           terms=KIN | POT):
    """wvl_apply_local_ham_static: the apply on the library's static
    workspace (no device allocation in the call); the plan's workspace must
    fit STATIC_WORKSPACE_BYTES (bound it with Plan(max_workspace=...))."""
    _need_cuda(psi_c, pot, hpsi_c, e_kin, e_pot)
    dt = _dtype_code(psi_c, pot, hpsi_c)
    _check_sizes(plan, psi_c, hpsi_c, e_kin, e_pot, None, dt)
    if pot is not None:
        n = plan.ctx.grid_n
        need = (2 * n[0] + 29) * (2 * n[1] + 29) * (2 * n[2] + 29)
        if pot.numel() != need:
            raise WvlError(WVL_EINVAL, f"potential has {pot.numel()} points, the grid needs {need}")
    _check(lib().wvl_apply_local_ham_static(plan._ptr, dt, int(terms), _ptr(psi_c), _ptr(pot),
                                           _ptr(hpsi_c), _ptr(e_kin), _ptr(e_pot)),
           plan.ctx.handle)


def kinetic(plan: Plan, psi_c, hpsi_c, e_kin=None, workspace=None):
    """wvl_kinetic: hpsi_c += L' T L psi_c."""
    _need_cuda(psi_c, hpsi_c, e_kin, workspace)
    dt = _dtype_code(psi_c, hpsi_c)
    _check_sizes(plan, psi_c, hpsi_c, e_kin, None, workspace, dt)
    if workspace is None:
        workspace = plan.new_workspace(psi_c.dtype)
    _check(lib().wvl_kinetic(plan._ptr, dt, _ptr(psi_c), _ptr(hpsi_c), _ptr(e_kin),
                            _ptr(workspace)), plan.ctx.handle)


def sparse_pattern_nnz(plan: Plan, ket_is_output: bool):
    n = ctypes.c_int64(0)
    _check(lib().wvl_sparse_overlap(plan._ptr, None, int(bool(ket_is_output)), None, F64,
                                   ctypes.byref(n), None, None, None), plan.ctx.handle)
    return n.value


def sparse_overlap(plan: Plan, bra_c, ket_c, ket_is_output: bool, out=None, values=True):
    """wvl_sparse_overlap -> (rowptr int64[nsf+1], col int32[nnz], val float64[nnz]),
    device tensors.  `out` may hold preallocated (rowptr, col, val); with
    values=False only the pattern is written (val is returned unfilled)."""
    import torch
    _need_cuda(bra_c, ket_c)
    dt = _dtype_code(bra_c, ket_c)
    if bra_c.numel() < plan.info["in_coefs"] or ket_c.numel() < plan.info[
            "out_coefs" if ket_is_output else "in_coefs"]:
        raise WvlError(WVL_EINVAL, "coefficient buffer smaller than the plan's layout")
    nnz = sparse_pattern_nnz(plan, ket_is_output)
    if out is None:
        rowptr = torch.empty(plan.nsf + 1, dtype=torch.int64, device="cuda")
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
        val = torch.empty(max(nnz, 1), dtype=torch.float64, device="cuda")
    else:
        rowptr, col, val = out
    n = ctypes.c_int64(0)
    _check(lib().wvl_sparse_overlap(plan._ptr, _ptr(bra_c), int(bool(ket_is_output)), _ptr(ket_c),
                                   dt, ctypes.byref(n), _ptr(rowptr), _ptr(col),
                                   _ptr(val) if values else None),
           plan.ctx.handle)
    return rowptr, col[:nnz], val[:nnz]


def gradient_scratch_bytes(plan: Plan):
    return 56 * max(1, sparse_pattern_nnz(plan, False))


def gradient(plan: Plan, s_val, h_val, k_val, psi_c, hpsi_c, g_c=None, scratch=None):
    """wvl_gradient: the localized support-function gradients (input layout)
    from S, H, the density kernel K (float64 device tensors in the CSR orders
    of the S / H patterns), psi_c and hpsi_c.  Returns g_c."""
    import torch
    _need_cuda(s_val, h_val, k_val, psi_c, hpsi_c, g_c, scratch)
    dt = _dtype_code(psi_c, hpsi_c) if g_c is None else _dtype_code(psi_c, hpsi_c, g_c)
    nnz_s, nnz_h = sparse_pattern_nnz(plan, False), sparse_pattern_nnz(plan, True)
    for t, n in ((s_val, nnz_s), (k_val, nnz_s), (h_val, nnz_h)):
        if t.dtype != torch.float64 or t.numel() < n:
            raise WvlError(WVL_EINVAL, "matrix values must be float64 on their pattern")
    if psi_c.numel() < plan.info["in_coefs"] or hpsi_c.numel() < plan.info["out_coefs"]:
        raise WvlError(WVL_EINVAL, "coefficient buffer smaller than the plan's layout")
    if g_c is None:
        g_c = torch.empty(max(1, plan.info["in_coefs"]), dtype=psi_c.dtype, device="cuda")
    if scratch is None:
        scratch = torch.empty(gradient_scratch_bytes(plan), dtype=torch.uint8, device="cuda")
    _check(lib().wvl_gradient(plan._ptr, dt, _ptr(s_val), _ptr(h_val), _ptr(k_val), _ptr(psi_c),
                             _ptr(hpsi_c), _ptr(g_c), _ptr(scratch),
                             scratch.numel() * scratch.element_size()), plan.ctx.handle)
    return g_c


def update(plan: Plan, psi_c, hpsi_c, h_val, eta):
    """wvl_update: psi_c <- psi_c - eta (P_L hpsi_c - H_aa psi_c), in place;
    h_val are the H values (float64, the plan's CSR order)."""
    _need_cuda(psi_c, hpsi_c, h_val)
    dt = _dtype_code(psi_c, hpsi_c)
    if psi_c.numel() < plan.info["in_coefs"] or hpsi_c.numel() < plan.info["out_coefs"]:
        raise WvlError(WVL_EINVAL, "coefficient buffer smaller than the plan's layout")
    if h_val.dtype.itemsize != 8 or h_val.numel() < sparse_pattern_nnz(plan, True):
        raise WvlError(WVL_EINVAL, "h_val must be float64 with the H pattern's nnz entries")
    _check(lib().wvl_update(plan._ptr, dt, float(eta), _ptr(hpsi_c), _ptr(h_val), _ptr(psi_c)),
           plan.ctx.handle)


def synthesize(plan: Plan, psi_c, fine, workspace=None):
    """wvl_synthesize: every function's real-space values on its fine box,
    concatenated in function order (plan.info["fine_box"] elements)."""
    _need_cuda(psi_c, fine, workspace)
    dt = _dtype_code(psi_c, fine)
    if psi_c.numel() < plan.info["in_coefs"] or fine.numel() < plan.info["fine_box"]:
        raise WvlError(WVL_EINVAL, "buffer smaller than the plan's layout")
    if workspace is None:
        workspace = plan.new_workspace(psi_c.dtype)
    _check(lib().wvl_synthesize(plan._ptr, dt, _ptr(psi_c), _ptr(fine), _ptr(workspace)),
           plan.ctx.handle)


def density(plan: Plan, fine, k_rowptr, k_col, k_val, rho, work=None):
    """wvl_density: rho (global fine grid, z, y, x) = sum_ab phi_a K^ab phi_b
    from the fine-box values `fine` and K in CSR form (int64 rowptr, int32
    col, float64 val, all on the device).  `work` is not used."""
    import torch
    _need_cuda(fine, k_rowptr, k_col, k_val, rho, work)
    dt = _dtype_code(fine, rho, work)
    n = plan.ctx.grid_n
    if rho.numel() < (2 * n[0] + 29) * (2 * n[1] + 29) * (2 * n[2] + 29):
        raise WvlError(WVL_EINVAL, "rho smaller than the fine grid")
    if fine.numel() < plan.info["fine_box"]:
        raise WvlError(WVL_EINVAL, "fine smaller than the plan's fine boxes")
    if k_rowptr.dtype != torch.int64 or k_rowptr.numel() < plan.nsf + 1 or \
            k_col.dtype != torch.int32 or k_val.dtype != torch.float64 or \
            k_col.numel() != k_val.numel():
        raise WvlError(WVL_EINVAL, "K must be CSR: int64 rowptr[nsf + 1], int32 col, float64 val")
    _check(lib().wvl_density(plan._ptr, dt, _ptr(fine), _ptr(k_rowptr), _ptr(k_col),
                             _ptr(k_val), int(k_val.numel()), _ptr(rho), _ptr(work)),
           plan.ctx.handle)


def foe_scratch_bytes(plan: Plan, npl, keep=True):
    """Scratch bytes of wvl_foe: with every Chebyshev matrix kept (one
    recursion), or the smaller size that runs the recursion twice."""
    nnz_s = sparse_pattern_nnz(plan, False)
    npl = max(1, int(npl))   # wvl_foe itself rejects npl < 1
    return 8 * ((npl + 7) * nnz_s + 2 * npl + 6) if keep else 8 * (9 * nnz_s + npl + 5)


def foe(plan: Plan, s_val, h_val, npl, delta, n_occ, eps_min=0.0, eps_max=0.0, k_val=None,
        scratch=None, keep=True):
    """wvl_foe: density kernel K on the overlap pattern by the Fermi operator
    expansion; returns (k_val, mu, e_bs).  s_val / h_val: float64 device
    values on the S / H patterns.  eps_min >= eps_max: Gershgorin bounds.
    Without a scratch buffer, one of foe_scratch_bytes(plan, npl, keep) is
    allocated; the library keeps the Chebyshev matrices when the buffer has
    room for them."""
    import torch
    _need_cuda(s_val, h_val, k_val, scratch)
    nnz_s, nnz_h = sparse_pattern_nnz(plan, False), sparse_pattern_nnz(plan, True)
    if s_val.dtype != torch.float64 or h_val.dtype != torch.float64 or \
            s_val.numel() < nnz_s or h_val.numel() < nnz_h:
        raise WvlError(WVL_EINVAL, "s_val / h_val must be float64 on the S / H patterns")
    if k_val is None:
        k_val = torch.empty(max(1, nnz_s), dtype=torch.float64, device="cuda")
    if scratch is None:
        scratch = torch.empty(foe_scratch_bytes(plan, npl, keep), dtype=torch.uint8,
                              device="cuda")
    mu, ebs = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().wvl_foe(plan._ptr, _ptr(s_val), _ptr(h_val), int(npl), float(delta),
                         float(n_occ), float(eps_min), float(eps_max), _ptr(k_val),
                         ctypes.byref(mu), ctypes.byref(ebs), _ptr(scratch),
                         scratch.numel() * scratch.element_size()), plan.ctx.handle)
    return k_val, mu.value, ebs.value


def precondition_scratch_bytes(plan: Plan, dtype_code):
    """Scratch bytes wvl_precondition needs (see include/wvl.h)."""
    sz = 8 if dtype_code == F64 else 4
    al = lambda n: (n + 255) // 256 * 256
    return 3 * al(plan.info["in_coefs"] * sz) + al(plan.info["out_coefs"] * sz) + \
        3 * al(8 * plan.nsf)


def precondition(plan: Plan, g_c, eps, niter, x_c, conf=None, workspace=None, scratch=None):
    """wvl_precondition: x_c <- approx. solution of (T + conf |r-R|^4 - eps) x = -g_c
    per function, `niter` conjugate-gradient steps; eps, conf float64 [nsf]."""
    import torch
    _need_cuda(g_c, x_c, eps, conf, workspace, scratch)
    dt = _dtype_code(g_c, x_c)
    if g_c.numel() < plan.info["in_coefs"] or x_c.numel() < plan.info["in_coefs"]:
        raise WvlError(WVL_EINVAL, "coefficient buffer smaller than the plan's layout")
    for v in (eps, conf):
        if v is not None and (v.dtype.itemsize != 8 or v.numel() < plan.nsf):
            raise WvlError(WVL_EINVAL, "eps / conf must be float64 with nsf entries")
    if workspace is None:
        workspace = plan.new_workspace(g_c.dtype)
    need = precondition_scratch_bytes(plan, dt)
    if scratch is None:
        scratch = torch.empty(need, dtype=torch.uint8, device="cuda")
    elif scratch.numel() * scratch.element_size() < need:
        raise WvlError(WVL_EINVAL, "scratch smaller than wvl_precondition needs")
    _check(lib().wvl_precondition(plan._ptr, dt, _ptr(g_c), _ptr(conf), _ptr(eps), int(niter),
                                  _ptr(x_c), _ptr(workspace), _ptr(scratch)), plan.ctx.handle)


class Graph:
    """One captured step (wvl_graph_create): the local-H apply of every
    function, then optionally the S values (into s_val) and the H values
    (into h_val) on the plan's patterns.  The tensors passed here must stay
    alive while the graph does; launch() replays the step on the context's
    stream."""

    def __init__(self, plan: Plan, psi_c, pot, hpsi_c, e_kin=None, e_pot=None, workspace=None,
                 s_val=None, h_val=None, terms=KIN | POT):
        _need_cuda(psi_c, pot, hpsi_c, e_kin, e_pot, workspace, s_val, h_val)
        dt = _dtype_code(psi_c, pot, hpsi_c)
        _check_sizes(plan, psi_c, hpsi_c, e_kin, e_pot, workspace, dt)
        for v, ket_out in ((s_val, False), (h_val, True)):
            if v is not None and (v.dtype.itemsize != 8 or
                                  v.numel() < sparse_pattern_nnz(plan, ket_out)):
                raise WvlError(WVL_EINVAL, "S/H value buffers must be float64 with nnz entries")
        if workspace is None:
            raise WvlError(WVL_EINVAL, "a graph needs an explicit workspace tensor")
        self.plan = plan
        self._keep = (psi_c, pot, hpsi_c, e_kin, e_pot, workspace, s_val, h_val)
        h = ctypes.c_void_p()
        _check(lib().wvl_graph_create(plan._ptr, dt, int(terms), _ptr(psi_c), _ptr(pot),
                                      _ptr(hpsi_c), _ptr(e_kin), _ptr(e_pot), _ptr(workspace),
                                      _ptr(s_val), _ptr(h_val), ctypes.byref(h)),
               plan.ctx.handle)
        self._ptr = h

    def launch(self):
        _check(lib().wvl_graph_launch(self._ptr), self.plan.ctx.handle)

    def close(self):
        if getattr(self, "_ptr", None):
            lib().wvl_graph_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_schedule(plan: Plan, nbins=1, kin_mfma=0):
    """wvl_plan_set_schedule: fix the plan's schedule (bins, z-kinetic form)."""
    _check(lib().wvl_plan_set_schedule(plan._ptr, int(nbins), int(kin_mfma)), plan.ctx.handle)
    plan.info = plan._read_info()


def autotune(plan: Plan, psi_c, pot, hpsi_c, workspace, reps=3, terms=KIN | POT):
    """wvl_plan_autotune -> (best, tried): dicts {nbins, kin_mfma, ms}."""
    _need_cuda(psi_c, pot, hpsi_c, workspace)
    dt = _dtype_code(psi_c, pot, hpsi_c)
    _check_sizes(plan, psi_c, hpsi_c, None, None, workspace, dt)
    tried = (_TunePoint * 32)()
    n = ctypes.c_int32(0)
    best = _TunePoint()
    _check(lib().wvl_plan_autotune(plan._ptr, dt, int(terms), _ptr(psi_c), _ptr(pot),
                                   _ptr(hpsi_c), _ptr(workspace), int(reps), tried, 32,
                                   ctypes.byref(n), ctypes.byref(best)), plan.ctx.handle)
    as_dict = lambda t: {"nbins": t.nbins, "kin_mfma": t.kin_mfma, "ms": t.ms}
    plan.info = plan._read_info()
    return as_dict(best), [as_dict(tried[i]) for i in range(n.value)]
