"""Approximate Kappa velocity generator for MI355X (gfx950).

Python binding of libkappa (include/kappa.h): an implementation of the
inverse-transform Kappa sampler of Zenitani & Umeda, "An approximate Kappa
generator for particle simulations" (arXiv 2602.05606, Table 1).  PyTorch is
used only to allocate device memory and to supply the HIP stream; every step
of the sampler runs in the library's HIP kernels.  There is no CPU fallback:
the functions raise if the library is missing or the device is not gfx950.

Precisions: FP64 (double outputs), FP32 (float outputs, FP32 bulk with an FP64
inversion when 1 - U1 < 2^-20) and FP32_NOTAIL (diagnostics).
"""
import ctypes

from . import _lib
from ._lib import FP32, FP32_NOTAIL, FP64, Cell, KappaError, Segment

__all__ = [
    "FP64", "FP32", "FP32_NOTAIL", "KappaError", "Segment", "params", "sample", "sample_backward",
    "KappaSample", "sample_backward_noalloc", "sample_autotune", "philox", "Plan", "sample_batched", "sample_exact_t", "sample_exact_pareto",
    "fill_probe", "copy_probe", "clock_probe", "clock_probe_stamps", "core_clock_hz", "issue_cost", "ISSUE_CLASSES",
    "transcendental_probe", "TRANSCENDENTALS", "backward_workspace_bytes", "version", "library_path", "speed_histogram",
    "relative_entropy", "divergence_grid", "optimum_c", "load_particles", "Cell", "SEGMENT_DTYPE", "segment_table",
]


def _torch():
    import torch
    return torch


def library_path():
    return _lib.LIB_PATH


def version():
    return _lib.load().kappa_version().decode()


def _dtype(precision):
    torch = _torch()
    return torch.float64 if precision == FP64 else torch.float32


def _raw_current_stream():
    """torch's raw current-stream query (no Stream object per call), or None."""
    torch = _torch()
    return getattr(torch._C, "_cuda_getCurrentRawStream", None)


_RAW_STREAM = None


def _stream(stream, device):
    """The HIP stream handle for a call: `stream`'s, or torch's current stream
    on `device` (a torch.device or a tensor's device)."""
    global _RAW_STREAM
    if stream is not None:
        return stream.cuda_stream
    if _RAW_STREAM is None:
        _RAW_STREAM = _raw_current_stream() or False
    torch = _torch()
    if _RAW_STREAM:
        index = device.index if isinstance(device, torch.device) else device
        return _RAW_STREAM(torch.cuda.current_device() if index is None else index)
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t):
    return t.data_ptr() if t is not None else None


def params(kappa):
    """Setup rows of Table 1 for one species (host FP64): dict with kstar, a,
    b, c, b_over_c, their kappa-derivatives da, db, dc, and lnbeta."""
    out = (ctypes.c_double * len(_lib.PARAM_NAMES))()
    _lib.check(_lib.load().kappa_params(float(kappa), out), "kappa_params")
    return dict(zip(_lib.PARAM_NAMES, list(out)))


def _outputs(n, precision, out, device):
    torch = _torch()
    if out is None:
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        return tuple(torch.empty(n, dtype=_dtype(precision), device=dev) for _ in range(3))
    vx, vy, vz = out
    for t in out:
        if t.dtype != _dtype(precision) or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
            raise ValueError("out tensors must be contiguous CUDA tensors of the precision's dtype and >= n elements")
    return vx, vy, vz


def sample(kappa, theta, n, seed, *, counter_offset=0, seg_id=0, precision=FP32, out=None, device=None,
           stream=None):
    """Particles counter_offset .. counter_offset+n-1 of segment seg_id.
    Returns (vx, vy, vz), device tensors (float64 for FP64, float32 otherwise)."""
    vx, vy, vz = _outputs(n, precision, out, device)
    st = _lib.load().kappa_sample(float(kappa), float(theta), n, seed, counter_offset, seg_id, precision,
                                  _ptr(vx), _ptr(vy), _ptr(vz), _stream(stream, vx.device))
    _lib.check(st, "kappa_sample")
    return vx, vy, vz


def sample_autotune(n, precision=FP32, reps=5, out=None, device=None, stream=None):
    """Times kappa_sample's launch shapes on n particles and keeps the fastest
    for this precision and size bucket (kappa_sample_autotune); returns
    (block, particles per thread)."""
    vx, vy, vz = _outputs(n, precision, out, device)
    b, u = ctypes.c_int(), ctypes.c_int()
    _lib.check(_lib.load().kappa_sample_autotune(precision, n, _ptr(vx), _ptr(vy), _ptr(vz), reps, ctypes.byref(b),
                                                 ctypes.byref(u), _stream(stream, vx.device)), "kappa_sample_autotune")
    return b.value, u.value


def backward_workspace_bytes(n):
    return int(_lib.load().kappa_backward_workspace_bytes(n))


def sample_backward(kappa, theta, n, seed, gx, gy, gz, *, counter_offset=0, seg_id=0, precision=FP32,
                    workspace=None, out=None, stream=None):
    """(dLoss/dkappa, dLoss/dtheta) through sample() at fixed uniforms, as a
    float64 device tensor of 2 elements (written into `out` when given).
    gx, gy, gz: upstream gradients."""
    torch = _torch()
    dev = gx.device
    dt = _dtype(precision)
    g = [t.contiguous() for t in (gx, gy, gz)]
    for t in g:
        if t.dtype != dt or t.numel() != n:
            raise ValueError(f"upstream gradients must be {dt} with {n} elements")
    wbytes = backward_workspace_bytes(n)
    if workspace is None:
        workspace = torch.empty(wbytes, dtype=torch.uint8, device=dev)
    grad = torch.empty(2, dtype=torch.float64, device=dev) if out is None else out
    if grad.dtype != torch.float64 or grad.numel() < 2 or not grad.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of at least 2 elements")
    st = _lib.load().kappa_sample_backward(float(kappa), float(theta), n, seed, counter_offset, seg_id, precision,
                                           _ptr(g[0]), _ptr(g[1]), _ptr(g[2]), _ptr(grad), _ptr(workspace),
                                           workspace.numel() * workspace.element_size(), _stream(stream, dev))
    _lib.check(st, "kappa_sample_backward")
    return grad


def sample_backward_noalloc(kappa, theta, n, seed, gx, gy, gz, grad, *, counter_offset=0, seg_id=0,
                            precision=FP32, stream=None):
    """sample_backward through kappa_sample_backward_noalloc: no workspace
    (the library's static per-device partial-sum array), and the result
    written into `grad` (a contiguous float64 device tensor of 2 elements,
    returned).  Calls that overlap on one device race on that array."""
    torch = _torch()
    dt = _dtype(precision)
    g = (gx, gy, gz)
    for t in g:
        if t.dtype != dt or t.numel() != n or not t.is_contiguous():
            raise ValueError(f"upstream gradients must be contiguous {dt} with {n} elements")
    if grad.dtype != torch.float64 or grad.numel() < 2 or not grad.is_contiguous():
        raise ValueError("grad must be a contiguous float64 tensor of at least 2 elements")
    st = _lib.load().kappa_sample_backward_noalloc(float(kappa), float(theta), n, seed, counter_offset, seg_id,
                                                   precision, _ptr(g[0]), _ptr(g[1]), _ptr(g[2]), _ptr(grad),
                                                   _stream(stream, gx.device))
    _lib.check(st, "kappa_sample_backward_noalloc")
    return grad


def _make_autograd():
    torch = _torch()

    class _KappaSample(torch.autograd.Function):
        """v = KappaSample.apply(kappa, theta, n, seed, counter_offset, seg_id, precision)

        kappa and theta are 0-d tensors; v is a (3, n) device tensor.  The
        backward pass returns dLoss/dkappa and dLoss/dtheta through the
        reparameterised sampler (the uniforms are fixed by seed and counters),
        computed by the library's backward kernel."""

        @staticmethod
        def forward(ctx, kappa, theta, n, seed, counter_offset=0, seg_id=0, precision=FP32):
            k, th = float(kappa), float(theta)
            dev = kappa.device if kappa.is_cuda else torch.device("cuda", torch.cuda.current_device())
            v = torch.empty((3, n), dtype=_dtype(precision), device=dev)
            sample(k, th, n, seed, counter_offset=counter_offset, seg_id=seg_id, precision=precision,
                   out=(v[0], v[1], v[2]))
            ctx.args = (k, th, n, seed, counter_offset, seg_id, precision)
            ctx.kappa_meta = (kappa.dtype, kappa.device, theta.dtype, theta.device)
            return v

        @staticmethod
        def backward(ctx, gv):
            k, th, n, seed, off, seg, prec = ctx.args
            gv = gv.to(_dtype(prec)).contiguous()
            grad = sample_backward(k, th, n, seed, gv[0], gv[1], gv[2], counter_offset=off, seg_id=seg,
                                   precision=prec)
            kd, kdev, td, tdev = ctx.kappa_meta
            return (grad[0].to(dtype=kd, device=kdev), grad[1].to(dtype=td, device=tdev),
                    None, None, None, None, None)

    return _KappaSample


KappaSample = _make_autograd()


def philox(n, seed, counter_offset=0, seg_id=0, draw=0, device=None, stream=None):
    """Raw Philox4x32-10 blocks as an (n, 4) int32 device tensor (the bits of
    the uint32 words r0..r3)."""
    torch = _torch()
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    out = torch.empty((n, 4), dtype=torch.int32, device=dev)
    st = _lib.load().kappa_philox(n, seed, counter_offset, seg_id, draw, _ptr(out), _stream(stream, dev))
    _lib.check(st, "kappa_philox")
    return out


def _segment_dtype():
    import numpy as np
    return np.dtype([("kappa", "<f8"), ("theta", "<f8"), ("drift", "<f8", (3,)), ("count", "<u8"),
                     ("seg_id", "<u4"), ("reserved", "<u4")], align=True)


def __getattr__(name):
    if name == "SEGMENT_DTYPE":  # numpy is imported only when the table form is used
        return _segment_dtype()
    raise AttributeError(name)


def segment_table(kappa, theta, count, seg_id=None, drift=None):
    """A segment table as a numpy structured array of SEGMENT_DTYPE (the
    kappa_segment layout), built from per-segment arrays without a Python loop:
    the form to use for plans of millions of segments.  seg_id defaults to
    0, 1, 2, ...; drift (shape (n, 3)) to zero."""
    import numpy as np
    kappa = np.asarray(kappa, dtype=np.float64)
    n = kappa.size
    t = np.zeros(n, dtype=_segment_dtype())
    t["kappa"] = kappa
    t["theta"] = np.broadcast_to(np.asarray(theta, dtype=np.float64), (n,))
    t["count"] = np.broadcast_to(np.asarray(count, dtype=np.uint64), (n,))
    t["seg_id"] = np.arange(n, dtype=np.uint32) if seg_id is None else np.asarray(seg_id, dtype=np.uint32)
    if drift is not None:
        t["drift"] = np.asarray(drift, dtype=np.float64).reshape(n, 3)
    return t


def _segments(segments):
    """Builds a ctypes array of Segment from Segment objects or dicts/tuples
    (kappa, theta, (dx, dy, dz), count, seg_id), or views a contiguous numpy
    array of SEGMENT_DTYPE (segment_table) without copying."""
    if type(segments).__module__ == "numpy" and getattr(segments, "dtype", None) == _segment_dtype():
        if not segments.flags["C_CONTIGUOUS"] or not segments.flags["WRITEABLE"]:
            raise ValueError("a segment table must be a contiguous, writeable numpy array")
        return (Segment * segments.size).from_buffer(segments)
    arr = (Segment * len(segments))()
    for i, s in enumerate(segments):
        if isinstance(s, Segment):
            arr[i] = s
            continue
        if isinstance(s, dict):
            kappa, theta, drift, count, seg_id = s["kappa"], s["theta"], s.get("drift", (0, 0, 0)), s["count"], s["seg_id"]
        else:
            kappa, theta, drift, count, seg_id = s
        arr[i].kappa = float(kappa)
        arr[i].theta = float(theta)
        arr[i].drift[0], arr[i].drift[1], arr[i].drift[2] = (float(d) for d in drift)
        arr[i].count = int(count)
        arr[i].seg_id = int(seg_id)
        arr[i].reserved = 0
    return arr


class Plan:
    """A batched plan (kappa_plan): many (species, cell) segments laid out back
    to back, sampled by one persistent kernel, optionally through a hipGraph."""

    def __init__(self, segments, seed, precision=FP32):
        self._segs = _segments(segments)
        self.precision = precision
        handle = ctypes.c_void_p()
        st = _lib.load().kappa_plan_create(self._segs, len(self._segs), seed, precision, ctypes.byref(handle))
        _lib.check(st, "kappa_plan_create")
        self._h = handle
        total = ctypes.c_uint64()
        _lib.check(_lib.load().kappa_plan_total(self._h, ctypes.byref(total)), "kappa_plan_total")
        self.total = total.value

    def outputs(self, device=None):
        return _outputs(self.total, self.precision, None, device)

    def launch(self, out, stream=None):
        vx, vy, vz = out
        _lib.check(_lib.load().kappa_plan_launch(self._h, _ptr(vx), _ptr(vy), _ptr(vz), _stream(stream, vx.device)),
                   "kappa_plan_launch")

    def graph_launch(self, out, stream=None):
        vx, vy, vz = out
        _lib.check(_lib.load().kappa_plan_graph_launch(self._h, _ptr(vx), _ptr(vy), _ptr(vz),
                                                       _stream(stream, vx.device)), "kappa_plan_graph_launch")

    def set_cells(self, cells):
        """One box per segment (in segment order) for fused particle loading:
        an array-like of shape (nseg, 2, 3) holding (lo, size), or None to
        remove the table (kappa_plan_set_cells)."""
        c = None if cells is None else _cells(cells, len(self._segs))
        _lib.check(_lib.load().kappa_plan_set_cells(self._h, c), "kappa_plan_set_cells")

    def launch_pic(self, pos, vel, stream=None):
        """Positions and velocities in one launch (kappa_plan_launch_pic)."""
        _lib.check(_lib.load().kappa_plan_launch_pic(self._h, *(_ptr(t) for t in pos), *(_ptr(t) for t in vel),
                                                     _stream(stream, vel[0].device)), "kappa_plan_launch_pic")

    def graph_launch_pic(self, pos, vel, stream=None):
        """launch_pic through the plan's captured hipGraph (kappa_plan_graph_launch_pic)."""
        _lib.check(_lib.load().kappa_plan_graph_launch_pic(self._h, *(_ptr(t) for t in pos),
                                                           *(_ptr(t) for t in vel), _stream(stream, vel[0].device)),
                   "kappa_plan_graph_launch_pic")

    def autotune(self, out, reps=5, stream=None):
        vx, vy, vz = out
        _lib.check(_lib.load().kappa_plan_autotune(self._h, _ptr(vx), _ptr(vy), _ptr(vz), reps,
                                                   _stream(stream, vx.device)), "kappa_plan_autotune")
        return self.shape

    @property
    def shape(self):
        b, u, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _lib.check(_lib.load().kappa_plan_shape(self._h, ctypes.byref(b), ctypes.byref(u), ctypes.byref(g)),
                   "kappa_plan_shape")
        return b.value, u.value, g.value

    def set_shape(self, block, unroll, grid):
        _lib.check(_lib.load().kappa_plan_set_shape(self._h, block, unroll, grid), "kappa_plan_set_shape")

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().kappa_plan_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _cells(cells, nseg):
    import numpy as np
    arr = np.asarray(cells, dtype=np.float64).reshape(-1, 2, 3)
    if arr.shape[0] != nseg:
        raise ValueError(f"{arr.shape[0]} cells for {nseg} segments")
    out = (_lib.Cell * nseg)()
    for s in range(nseg):
        out[s].lo[:] = arr[s, 0].tolist()
        out[s].size[:] = arr[s, 1].tolist()
    return out


def load_particles(segments, cells, seed, precision=FP32, device=None, stream=None):
    """One-shot fused particle loading (kappa_load_particles, synchronous):
    returns ((px, py, pz), (vx, vy, vz)).  cells: (nseg, 2, 3) of (lo, size)."""
    segs = _segments(segments)
    total = sum(int(s.count) for s in segs)
    pos = _outputs(total, precision, None, device)
    vel = _outputs(total, precision, None, device)
    st = _lib.load().kappa_load_particles(segs, _cells(cells, len(segs)), len(segs), seed, precision,
                                          *(_ptr(t) for t in pos), *(_ptr(t) for t in vel),
                                          _stream(stream, vel[0].device))
    _lib.check(st, "kappa_load_particles")
    return pos, vel


def sample_batched(segments, seed, precision=FP32, out=None, device=None, stream=None):
    """One-shot batched sampling (kappa_sample_batched, synchronous)."""
    segs = _segments(segments)
    if type(segments).__module__ == "numpy":
        total = int(segments["count"].sum(dtype="u8"))
    else:
        total = sum(int(s.count) for s in segs)
    vx, vy, vz = _outputs(total, precision, out, device)
    st = _lib.load().kappa_sample_batched(segs, len(segs), seed, precision, _ptr(vx), _ptr(vy), _ptr(vz),
                                          _stream(stream, vx.device))
    _lib.check(st, "kappa_sample_batched")
    return vx, vy, vz


def _exact(fn_name, kappa, theta, n, seed, precision, with_iters, out, device, stream):
    torch = _torch()
    vx, vy, vz = _outputs(n, precision, out, device)
    iters = torch.empty(n, dtype=torch.int32, device=vx.device) if with_iters else None
    st = getattr(_lib.load(), fn_name)(float(kappa), float(theta), n, seed, precision, _ptr(vx), _ptr(vy), _ptr(vz),
                                       _ptr(iters), _stream(stream, vx.device))
    _lib.check(st, fn_name)
    return (vx, vy, vz, iters) if with_iters else (vx, vy, vz)


def sample_exact_t(kappa, theta, n, seed, precision=FP32, with_iters=False, out=None, device=None, stream=None):
    """Exact Kappa samples via 3 normals / sqrt(Gamma(kappa - 1/2)) (comparator)."""
    return _exact("kappa_sample_exact_t", kappa, theta, n, seed, precision, with_iters, out, device, stream)


def sample_exact_pareto(kappa, theta, n, seed, precision=FP32, with_iters=False, out=None, device=None, stream=None):
    """Exact Kappa samples via Type II Pareto acceptance-rejection (comparator)."""
    return _exact("kappa_sample_exact_pareto", kappa, theta, n, seed, precision, with_iters, out, device, stream)


def fill_probe(n, precision, out, stream=None):
    vx, vy, vz = out
    _lib.check(_lib.load().kappa_fill_probe(n, precision, _ptr(vx), _ptr(vy), _ptr(vz), _stream(stream, vx.device)),
               "kappa_fill_probe")


def copy_probe(src, dst, stream=None):
    nbytes = src.numel() * src.element_size()
    _lib.check(_lib.load().kappa_copy_probe(_ptr(src), _ptr(dst), nbytes, _stream(stream, src.device)),
               "kappa_copy_probe")


def clock_probe(kappa, theta, n, seed, *, counter_offset=0, seg_id=0, precision=FP32, out=None, device=None,
                stamps=None, stream=None):
    """sample() through kappa_clock_probe: the same outputs from the same
    kernel, plus per-workgroup clock stamps.  Returns ((vx, vy, vz), stamps,
    wall_hz) with stamps an int64 device tensor of shape (workgroups, 4):
    shader-clock counter at entry, constant-rate counter at entry, the same
    two at exit; the constant-rate counter ticks at wall_hz.  `stamps` may
    bring a contiguous int64 device buffer (clock_probe_stamps(n) entries)."""
    torch = _torch()
    vx, vy, vz = _outputs(n, precision, out, device)
    if stamps is None:
        stamps = torch.empty(clock_probe_stamps(n), dtype=torch.int64, device=vx.device)
    elif stamps.dtype != torch.int64 or not stamps.is_contiguous():
        raise ValueError("stamps must be a contiguous int64 device tensor")
    blocks, hz = ctypes.c_uint32(0), ctypes.c_double(0.0)
    st = _lib.load().kappa_clock_probe(float(kappa), float(theta), n, seed, counter_offset, seg_id, precision,
                                       _ptr(vx), _ptr(vy), _ptr(vz), _ptr(stamps), stamps.numel(),
                                       ctypes.byref(blocks), ctypes.byref(hz), _stream(stream, vx.device))
    _lib.check(st, "kappa_clock_probe")
    return (vx, vy, vz), stamps[:4 * blocks.value].view(blocks.value, 4), hz.value


def clock_probe_stamps(n):
    """Entries of a stamps buffer that suffices for clock_probe of n particles."""
    return 4 * max(1, -(-n // 64))


ISSUE_CLASSES = {"fma_f32": 0, "transcendental_f32": 1, "mad_u64_u32": 2, "fma_f64": 3, "bitop3_b32": 4,
                 "log_plus_3fma_f32": 5, "fma_f32_literal": 6}


def issue_cost(op, reps=5, device=None, stream=None):
    """SIMD-cycles per wave64 instruction of one instruction class
    (kappa_issue_probe; op a key or value of ISSUE_CLASSES), from reps
    back-to-back launches timed with events and the core clock of the last
    one.  Returns {"cycles": ..., "clock_ghz": ...}."""
    torch = _torch()
    op = ISSUE_CLASSES.get(op, op)
    lib = _lib.load()
    blocks, steps, hz = ctypes.c_uint32(0), ctypes.c_uint32(0), ctypes.c_double(0.0)
    st = lib.kappa_issue_probe(op, None, 0, None, 0, ctypes.byref(blocks), ctypes.byref(steps), ctypes.byref(hz),
                               None)
    if st != _lib.ERANGE:
        _lib.check(st, "kappa_issue_probe")
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    sink = torch.empty(blocks.value * 256, dtype=torch.float32, device=dev)
    stamps = torch.empty(blocks.value * 8, dtype=torch.int64, device=dev)
    s = _stream(stream, dev)

    def launch():
        _lib.check(lib.kappa_issue_probe(op, _ptr(sink), sink.numel(), _ptr(stamps), stamps.numel(),
                                         ctypes.byref(blocks), ctypes.byref(steps), ctypes.byref(hz), s),
                   "kappa_issue_probe")

    for _ in range(2):
        launch()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        launch()
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    h = stamps.cpu()
    clock = int(h[0::2].sum()) / int(h[1::2].sum()) * hz.value
    simds = blocks.value // 2  # 8 workgroups per CU, 4 SIMDs per CU
    return {"cycles": simds * clock * sec / (4 * blocks.value * steps.value), "clock_ghz": clock / 1e9}


TRANSCENDENTALS = {"log2": 0, "exp2": 1, "sin_rev": 2, "cos_rev": 3, "sqrt": 4, "rsq": 5, "rcp": 6}


def transcendental_probe(op, x, out=None, stream=None):
    """The gfx950 hardware instruction applied to each element of the float32
    device tensor x (kappa_transcendental_probe; op a key or value of
    TRANSCENDENTALS; sin_rev and cos_rev take revolutions)."""
    torch = _torch()
    op = TRANSCENDENTALS.get(op, op)
    x = x.contiguous()
    if x.dtype != torch.float32:
        raise ValueError("x must be float32")
    out = torch.empty_like(x) if out is None else out
    _lib.check(_lib.load().kappa_transcendental_probe(op, _ptr(x), _ptr(out), x.numel(), _stream(stream, x.device)),
               "kappa_transcendental_probe")
    return out


def core_clock_hz(stamps, wall_hz):
    """Mean core clock (Hz) over the waves stamped by clock_probe, each weighted
    by its duration: total core cycles over total constant-rate time."""
    s = stamps.cpu()
    cycles = int((s[:, 2] - s[:, 0]).sum())  # differences in int64: the counters run from boot
    ticks = int((s[:, 3] - s[:, 1]).sum())
    return cycles / ticks * wall_hz if ticks > 0 else float("nan")


def speed_histogram(vx, vy, vz, theta, bin_width=0.2, nbins=100, counts=None, stream=None):
    """Counts of |v| in bins [k w theta, (k+1) w theta), k < nbins, plus an
    overflow bin (kappa_speed_histogram).  counts (int64 device tensor of
    nbins + 1) is accumulated when given; a new zeroed one otherwise."""
    torch = _torch()
    n = vx.numel()
    prec = FP64 if vx.dtype == torch.float64 else FP32
    if counts is None:
        counts = torch.zeros(nbins + 1, dtype=torch.int64, device=vx.device)
    st = _lib.load().kappa_speed_histogram(_ptr(vx), _ptr(vy), _ptr(vz), n, prec, float(theta), float(bin_width),
                                           nbins, _ptr(counts), _stream(stream, vx.device))
    _lib.check(st, "kappa_speed_histogram")
    return counts


def divergence_grid(kappa, c=None, energy=True, argmin=False, device=None, stream=None):
    """Relative entropy D(f||g; kappa, c) (eq:relative_entropy) and energy
    error (E_approx - E_kappa)/E_kappa (Fig. fig:DE(b)) of the approximation
    on the grid kappa x c (kappa_divergence_grid).  kappa and c are 1-D
    sequences or float64 device tensors; c=None takes c from eq:c for each
    kappa (one column).  Returns (D, dE or None, argmin or None) as device
    tensors of shape (nk, nc), (nk, nc) and (nk,)."""
    torch = _torch()
    dev = torch.device(device) if device is not None else (
        kappa.device if hasattr(kappa, "device") and kappa.is_cuda else torch.device("cuda"))
    k = torch.as_tensor(kappa, dtype=torch.float64, device=dev).contiguous().reshape(-1)
    cv = None if c is None else torch.as_tensor(c, dtype=torch.float64, device=dev).contiguous().reshape(-1)
    nk, nc = k.numel(), (1 if cv is None else cv.numel())
    D = torch.empty((nk, nc), dtype=torch.float64, device=dev)
    dE = torch.empty((nk, nc), dtype=torch.float64, device=dev) if energy else None
    am = torch.empty(nk, dtype=torch.int32, device=dev) if argmin else None
    st = _lib.load().kappa_divergence_grid(_ptr(k), nk, _ptr(cv), nc, _ptr(D), _ptr(dE), _ptr(am),
                                           _stream(stream, dev))
    _lib.check(st, "kappa_divergence_grid")
    return D, dE, am


def optimum_c(kappa, c_grid, iters=40, device=None, stream=None):
    """The c minimising D(f||g; kappa, c) for each kappa: the grid search of
    Sec. 3 over c_grid (ascending), refined by golden-section steps between the
    grid neighbours of the best point (kappa_optimum_c).  Returns (c_opt, D_opt)
    as float64 device tensors of shape (nk,)."""
    torch = _torch()
    dev = torch.device(device) if device is not None else (
        kappa.device if hasattr(kappa, "device") and kappa.is_cuda else torch.device("cuda"))
    k = torch.as_tensor(kappa, dtype=torch.float64, device=dev).contiguous().reshape(-1)
    cg = torch.as_tensor(c_grid, dtype=torch.float64, device=dev).contiguous().reshape(-1)
    c_opt = torch.empty(k.numel(), dtype=torch.float64, device=dev)
    d_opt = torch.empty(k.numel(), dtype=torch.float64, device=dev)
    st = _lib.load().kappa_optimum_c(_ptr(k), k.numel(), _ptr(cg), cg.numel(), iters, _ptr(c_opt), _ptr(d_opt),
                                     _stream(stream, dev))
    _lib.check(st, "kappa_optimum_c")
    return c_opt, d_opt


def relative_entropy(kappa, counts, bin_width=0.2, eps=1e-10, with_probabilities=False):
    """The paper's Monte Carlo relative entropy (eq:KL) of a speed histogram
    (nbins + 1 counts, the last bin open-ended; a torch tensor or any array)
    through kappa_relative_entropy: D(P||Q) = sum_i (P_i + eps) ln((P_i + eps)
    / (Q_i + eps)), P_i the exact Kappa probability of speed bin i (width
    bin_width in units of theta), Q_i the fraction of the counts.  With
    with_probabilities, returns (D, P) with P the exact bin probabilities."""
    import numpy as np
    c = counts.detach().cpu().numpy() if hasattr(counts, "detach") else np.asarray(counts)
    c = np.ascontiguousarray(np.rint(c).astype(np.uint64) if c.dtype.kind == "f" else c.astype(np.uint64))
    nb = c.size - 1
    d = ctypes.c_double()
    p = np.empty(nb + 1, dtype=np.float64)
    _lib.check(_lib.load().kappa_relative_entropy(float(kappa), c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), nb,
                                                  float(bin_width), float(eps), ctypes.byref(d),
                                                  p.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "kappa_relative_entropy")
    return (d.value, p) if with_probabilities else d.value
