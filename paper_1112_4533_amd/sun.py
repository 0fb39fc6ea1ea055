"""Python binding of libsun (include/sun.h): argument marshalling only.

Device memory comes from PyTorch (uint8 tensors on the current CUDA/HIP
device) and every call is queued on torch's current stream.  All work runs in
the HIP kernels of libsun; there is no CPU fallback: if the library is not
built, load() raises.
"""
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libsun.so")

F32, F64, F32_TWO_ROW, F64_TWO_ROW, F32_WIDE, F64_WIDE = 0, 1, 2, 3, 4, 5
DTYPE_NAMES = {F32: "f32", F64: "f64", F32_TWO_ROW: "f32r12", F64_TWO_ROW: "f64r12", F32_WIDE: "f32w",
               F64_WIDE: "f64w"}
NC_MAX_REGISTER, NC_MAX = 4, 32
HEATBATH, OVERRELAX = 0, 1
KERNEL_IDS = {"heatbath": 0, "overrelax": 1, "reunit": 2, "plaquette": 3, "polyakov": 4}
SUN_OK, SUN_EINVAL, SUN_ESIZE, SUN_EHIP, SUN_EUNSUP, SUN_ENUMERIC = 0, -1, -2, -3, -4, -5

_lib = None


class SunError(RuntimeError):
    """A libsun call failed; `code` is its SUN_E* status."""

    def __init__(self, msg, code=None):
        super().__init__(msg)
        self.code = code


class SunNumericError(SunError):
    """The watchdog found a non-finite or non-unitary field (SUN_ENUMERIC)."""


def load():
    """Loads libsun.so (after torch, so both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SunError(f"{LIB_PATH} is missing: build it with paper_1112_4533_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    c_int, c_u64, c_u32, c_dbl, vp = ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p
    L4 = ctypes.c_int * 4
    sz = ctypes.c_size_t
    sigs = {
        "sun_lattice_bytes": [c_int, L4, c_int, ctypes.POINTER(sz), ctypes.POINTER(sz)],
        "sun_lattice_create": [c_int, L4, c_int, vp, sz, vp, sz, ctypes.POINTER(vp)],
        "sun_init": [vp, c_int, c_u64, vp],
        "sun_phase": [vp, c_int, c_int, c_int, c_dbl, c_u64, c_u64, vp],
        "sun_sweep": [vp, c_dbl, c_int, c_int, c_u64, c_int, vp],
        "sun_reunitarize": [vp, vp, vp],
        "sun_plaquette": [vp, vp, vp],
        "sun_polyakov": [vp, vp, vp],
        "sun_unitarity": [vp, vp, vp],
        "sun_watchdog": [vp, c_dbl, vp],
        "sun_check": [vp, ctypes.POINTER(c_dbl), vp],
        "sun_export": [vp, vp, vp],
        "sun_import": [vp, vp, vp],
        "sun_get_step": [vp, ctypes.POINTER(c_u64)],
        "sun_set_step": [vp, c_u64],
        "sun_profile": [vp, c_int],
        "sun_profile_read": [vp, c_int, ctypes.POINTER(c_dbl), ctypes.POINTER(ctypes.c_int64)],
        "sun_sample_su2": [c_int, vp, c_int, c_u64, c_u32, c_u32, vp, vp, vp],
        "sun_batch_bytes": [c_int, ctypes.POINTER(sz)],
        "sun_batch_create": [c_int, ctypes.POINTER(vp), ctypes.POINTER(c_dbl), ctypes.POINTER(c_u64), vp, sz,
                             ctypes.POINTER(vp)],
        "sun_batch_sweep": [vp, c_int, c_int, c_int, vp, vp],
        "sun_batch_plaquette": [vp, vp, vp],
        "sun_batch_capture": [vp, c_int, c_int, c_int, c_int, vp, vp, vp],
        "sun_batch_replay": [vp, vp],
        "sun_batch_sync": [vp],
        "sun_set_launch": [vp, c_int, c_int, c_int, c_int, c_int],
        "sun_get_launch": [vp, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                           ctypes.POINTER(c_int)],
        "sun_batch_set_launch": [vp, c_int, c_int, c_int, c_int],
        "sun_set_sites_per_item": [vp, c_int, c_int],
        "sun_get_sites_per_item": [vp, c_int, ctypes.POINTER(c_int)],
        "sun_batch_set_sites_per_item": [vp, c_int, c_int],
        "sun_plaquette_static": [c_int, L4, c_int, vp, vp, vp],
        "sun_set_tile_order": [vp, c_u64],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = c_int
    L.sun_lattice_destroy.argtypes = [vp]
    L.sun_lattice_destroy.restype = None
    L.sun_batch_destroy.argtypes = [vp]
    L.sun_batch_destroy.restype = None
    L.sun_last_error.argtypes = []
    L.sun_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def exported_symbols():
    """Names declared in include/sun.h that libsun exports."""
    L = load()
    return [n for n in ("sun_lattice_bytes", "sun_lattice_create", "sun_lattice_destroy", "sun_init",
                        "sun_phase", "sun_sweep", "sun_reunitarize", "sun_plaquette", "sun_polyakov",
                        "sun_unitarity", "sun_watchdog", "sun_check", "sun_export", "sun_import", "sun_get_step", "sun_set_step",
                        "sun_profile", "sun_profile_read", "sun_sample_su2", "sun_last_error",
                        "sun_batch_bytes", "sun_batch_create", "sun_batch_sweep", "sun_batch_plaquette",
                        "sun_batch_capture", "sun_batch_replay", "sun_batch_sync", "sun_batch_destroy",
                        "sun_set_launch", "sun_get_launch", "sun_batch_set_launch", "sun_set_sites_per_item",
                        "sun_get_sites_per_item", "sun_batch_set_sites_per_item", "sun_plaquette_static",
                        "sun_set_tile_order")
            if hasattr(L, n)]


def _check(rc):
    if rc != SUN_OK:
        cls = SunNumericError if rc == SUN_ENUMERIC else SunError
        raise cls(f"libsun error {rc}: {load().sun_last_error().decode()}", rc)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dtype_code(dtype):
    """Link storage: "f32", "f64", the SU(3) two-row forms "f32r12",
    "f64r12", or "f32w", "f64w" for the workgroup-per-link path at any
    Nc >= 4 (which "f32" / "f64" select by themselves above Nc = 4); also the
    integer codes."""
    if isinstance(dtype, int) and dtype in DTYPE_NAMES:
        return dtype
    if dtype in ("f32", "float32", torch.float32):
        return F32
    if dtype in ("f64", "float64", torch.float64):
        return F64
    for code, name in DTYPE_NAMES.items():
        if dtype == name:
            return code
    raise ValueError(f"unknown link dtype {dtype!r}")


def lattice_bytes(nc, L, dtype="f32"):
    lb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load().sun_lattice_bytes(int(nc), (ctypes.c_int * 4)(*L), _dtype_code(dtype), ctypes.byref(lb),
                                    ctypes.byref(sb)))
    return lb.value, sb.value


class Lattice:
    """An SU(Nc) gauge field on an L[0] x L[1] x L[2] x L[3] periodic lattice,
    stored on the GPU in the library's SoA layout."""

    def __init__(self, nc, L, dtype="f32", device=None):
        self.nc = int(nc)
        self.L = tuple(int(v) for v in L)
        self.dtype = _dtype_code(dtype)
        self.V = 1
        for v in self.L:
            self.V *= v
        lib = load()
        lb, sb = lattice_bytes(self.nc, self.L, self.dtype)
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.links = torch.empty(lb, dtype=torch.uint8, device=dev)
        self.scratch = torch.empty(sb, dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p()
        _check(lib.sun_lattice_create(self.nc, (ctypes.c_int * 4)(*self.L), self.dtype, _ptr(self.links), lb,
                                      _ptr(self.scratch), sb, ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.sun_lattice_destroy(h)
            self._h = None

    # -- updates ---------------------------------------------------------
    def init(self, hot=True, seed=0):
        _check(load().sun_init(self._h, int(bool(hot)), int(seed), _stream()))

    def phase(self, kind, mu, parity, beta, seed, step):
        _check(load().sun_phase(self._h, int(kind), int(mu), int(parity), float(beta), int(seed), int(step),
                                _stream()))

    def sweep(self, beta, n_hb=1, n_or=4, seed=0, reunit=True):
        _check(load().sun_sweep(self._h, float(beta), int(n_hb), int(n_or), int(seed), int(bool(reunit)),
                                _stream()))

    def phase_step(self, kind, beta=1.0, seed=0, step=0):
        """All eight phases (mu = 0..3, even then odd) of one update kind,
        leaving the RNG step counter alone."""
        for mu in range(4):
            for p in range(2):
                self.phase(kind, mu, p, beta, seed, step)

    def reunitarize(self, report=False):
        """Returns a device tensor {max|U^dag U - 1|, max|det - 1|} measured
        before the projection when report is true."""
        out = torch.zeros(2, dtype=torch.float64, device=self.links.device) if report else None
        _check(load().sun_reunitarize(self._h, _ptr(out) if report else None, _stream()))
        return out

    # -- measurements (device tensors, asynchronous) ---------------------
    def plaquette(self, out=None):
        out = out if out is not None else torch.empty(3, dtype=torch.float64, device=self.links.device)
        _check(load().sun_plaquette(self._h, _ptr(out), _stream()))
        return out

    def polyakov(self, out=None):
        out = out if out is not None else torch.empty(2, dtype=torch.float64, device=self.links.device)
        _check(load().sun_polyakov(self._h, _ptr(out), _stream()))
        return out

    def unitarity(self, out=None):
        out = out if out is not None else torch.empty(2, dtype=torch.float64, device=self.links.device)
        _check(load().sun_unitarity(self._h, _ptr(out), _stream()))
        return out

    # -- watchdog ---------------------------------------------------------
    def watchdog(self, threshold):
        """Arms (threshold > 0) or disarms (0) the check made by every later
        re-unitarization (reunitarize(), and sweep() with reunit), and clears
        its state."""
        _check(load().sun_watchdog(self._h, float(threshold), _stream()))

    def check(self):
        """Waits for the queued work; raises SunNumericError if a check since
        watchdog() tripped, else returns 0.0."""
        d = ctypes.c_double()
        _check(load().sun_check(self._h, ctypes.byref(d), _stream()))
        return d.value

    # -- field transfer --------------------------------------------------
    def export(self):
        """Canonical FP64 field as a (4, V, Nc, Nc) complex128 device tensor."""
        out = torch.empty((4, self.V, self.nc, self.nc, 2), dtype=torch.float64, device=self.links.device)
        _check(load().sun_export(self._h, _ptr(out), _stream()))
        return torch.view_as_complex(out)

    def import_(self, field):
        """Loads a canonical (4, V, Nc, Nc) complex field (device or host)."""
        t = torch.as_tensor(field)
        assert tuple(t.shape) == (4, self.V, self.nc, self.nc), t.shape
        t = torch.view_as_real(t.to(torch.complex128)).contiguous().to(self.links.device)
        _check(load().sun_import(self._h, _ptr(t), _stream()))
        torch.cuda.current_stream().synchronize()

    @property
    def step(self):
        v = ctypes.c_uint64()
        _check(load().sun_get_step(self._h, ctypes.byref(v)))
        return v.value

    @step.setter
    def step(self, value):
        _check(load().sun_set_step(self._h, int(value)))

    # -- launch shape (tuning only; results do not depend on it) ---------
    # (work-items per workgroup, XCD-aware order, resident-wave cap per CU,
    #  time slices per block of the tile walk)
    LAUNCH_SHAPES = [(b, x, w, t) for b in (64, 128, 256) for x in (1, 0) for w in (8, 12, 16, 0)
                     for t in (0, 2, 4, 8)]

    def set_launch(self, block=256, xcd=1, waves=0, tblock=0, kind=-1):
        """Launch shape of the heatbath (kind 0), overrelaxation (1) or both
        (-1) phase kernels.  On the workgroup-per-link path (Nc >= 5, or the
        WIDE storages) only the block applies: 64 or 128 threads per link
        (one or two wavefronts), any other value the library's choice."""
        _check(load().sun_set_launch(self._h, int(kind), int(block), int(xcd), int(waves), int(tblock)))

    def get_launch(self, kind):
        """(block, xcd, waves, tblock in effect) of one update kind."""
        b, x, w, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(load().sun_get_launch(self._h, int(kind), ctypes.byref(b), ctypes.byref(x), ctypes.byref(w),
                                     ctypes.byref(t)))
        return b.value, x.value, w.value, t.value

    @property
    def launch(self):
        """(heatbath shape, overrelaxation shape)."""
        return self.get_launch(HEATBATH), self.get_launch(OVERRELAX)

    SITES_PER_ITEM = (1, 2, 4)

    def set_sites_per_item(self, spt, kind=-1):
        """Sites each work-item of the phase kernels updates in turn (1, 2
        or 4), for kind 0, 1 or both (-1)."""
        _check(load().sun_set_sites_per_item(self._h, int(kind), int(spt)))

    def get_sites_per_item(self, kind):
        v = ctypes.c_int()
        _check(load().sun_get_sites_per_item(self._h, int(kind), ctypes.byref(v)))
        return v.value

    def set_tile_order(self, seed):
        """Random tile order per phase (race check; 0 restores the default)."""
        _check(load().sun_set_tile_order(self._h, int(seed)))

    # -- event timing ----------------------------------------------------
    def profile(self, enable=True, every=1):
        """Starts (or with enable=False stops) event timing of one launch in
        `every` per kernel kind; clears the totals."""
        _check(load().sun_profile(self._h, int(every) if enable else 0))

    def profile_read(self, kernel):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(load().sun_profile_read(self._h, KERNEL_IDS.get(kernel, kernel), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


class Batch:
    """Independent chains advanced together: one launch per phase and per
    (Nc, precision) group, optionally replayed from a captured HIP graph.
    The lattices keep their fields; while the batch is in use they should be
    driven only through it (sync() hands the step counters back)."""

    # (work-items per workgroup, XCD-aware order, resident-wave cap per CU);
    # batches always walk their tiles linearly
    LAUNCH_SHAPES = [(b, x, w) for b in (64, 128, 256) for x in (1, 0) for w in (8, 12, 16, 0)]

    def __init__(self, lattices, betas, seeds):
        self.lattices = list(lattices)
        n = len(self.lattices)
        assert n > 0 and len(betas) == n and len(seeds) == n
        lib = load()
        tb = ctypes.c_size_t()
        _check(lib.sun_batch_bytes(n, ctypes.byref(tb)))
        dev = self.lattices[0].links.device
        self.table = torch.empty(tb.value, dtype=torch.uint8, device=dev)
        handles = (ctypes.c_void_p * n)(*[l._h.value for l in self.lattices])
        b = (ctypes.c_double * n)(*[float(x) for x in betas])
        sd = (ctypes.c_uint64 * n)(*[int(x) for x in seeds])
        h = ctypes.c_void_p()
        _check(lib.sun_batch_create(n, handles, b, sd, _ptr(self.table), tb.value, ctypes.byref(h)))
        self._h = h
        self.n = n
        self.betas = [float(x) for x in betas]
        self.seeds = [int(x) for x in seeds]
        self.launch = [(256, 1, 0), (256, 1, 0)]    # heatbath, overrelaxation (block, xcd, waves)
        self.sites_per_item = [1, 1]
        self.stream = torch.cuda.Stream(device=dev)   # graphs need a non-null stream

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.sun_batch_destroy(h)
            self._h = None

    def sweep(self, n_hb=1, n_or=4, reunit=True, beta=None):
        """One sweep of every chain; beta: None (the couplings in force), or an
        (n,) float64 device tensor of couplings in chain order."""
        _check(load().sun_batch_sweep(self._h, int(n_hb), int(n_or), int(bool(reunit)),
                                      _ptr(beta) if beta is not None else None, _stream()))

    def plaquette(self, out=None):
        out = out if out is not None else torch.empty((self.n, 3), dtype=torch.float64,
                                                      device=self.table.device)
        _check(load().sun_batch_plaquette(self._h, _ptr(out), _stream()))
        return out

    def capture(self, n_sweeps=1, n_hb=1, n_or=4, reunit=True, plaq_out=None, beta=None):
        """Captures n_sweeps sweeps (plus plaquettes into plaq_out, an (n, 3)
        float64 device tensor, if given) as one graph; with beta (an (n,)
        float64 device tensor) each replay takes the couplings it holds then."""
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        _check(load().sun_batch_capture(self._h, int(n_sweeps), int(n_hb), int(n_or), int(bool(reunit)),
                                        _ptr(beta) if beta is not None else None,
                                        _ptr(plaq_out) if plaq_out is not None else None,
                                        ctypes.c_void_p(self.stream.cuda_stream)))

    def replay(self):
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        _check(load().sun_batch_replay(self._h, ctypes.c_void_p(self.stream.cuda_stream)))
        cur.wait_stream(self.stream)

    def sync(self):
        _check(load().sun_batch_sync(self._h))

    def set_launch(self, block=256, xcd=1, waves=0, kind=-1):
        """Launch shape of the phase kernels (kind as Lattice.set_launch);
        drops a captured graph."""
        _check(load().sun_batch_set_launch(self._h, int(kind), int(block), int(xcd), int(waves)))
        for k in ((HEATBATH, OVERRELAX) if kind < 0 else (kind,)):
            self.launch[k] = (int(block), int(xcd), int(waves))

    def set_sites_per_item(self, spt, kind=-1):
        """Sites per work-item of the phase kernels (as Lattice); drops a
        captured graph."""
        _check(load().sun_batch_set_sites_per_item(self._h, int(kind), int(spt)))
        for k in ((HEATBATH, OVERRELAX) if kind < 0 else (kind,)):
            self.sites_per_item[k] = int(spt)


def plaquette_static(nc, L, dtype, links, out=None):
    """The plaquette of a field in caller memory (a lattice's `links`
    tensor, or any buffer of that layout) through sun_plaquette_static: no
    handle and no allocation inside the library; `out` (3 float64 on the
    device) is allocated here if not given."""
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=links.device)
    _check(load().sun_plaquette_static(int(nc), (ctypes.c_int * 4)(*L), _dtype_code(dtype), _ptr(links), _ptr(out),
                                       _stream()))
    return out


def sample_su2(alpha, seed, step=0, mu_sg=0, dtype="f64"):
    """SU(2) heatbath draws on the GPU for a device float64 tensor alpha."""
    alpha = alpha.to(torch.float64).contiguous()
    n = alpha.numel()
    x = torch.empty((n, 4), dtype=torch.float64, device=alpha.device)
    att = torch.empty(n, dtype=torch.int32, device=alpha.device)
    _check(load().sun_sample_su2(_dtype_code(dtype), _ptr(alpha), n, int(seed), int(step), int(mu_sg), _ptr(x),
                                 _ptr(att), _stream()))
    return x, att
