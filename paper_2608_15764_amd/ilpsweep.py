"""ctypes binding of the C ABI in ``include/ilpsweep.h``.

Argument marshalling only: every step of the path runs in the HIP kernels of
``libilpsweep.so``.  Device pointers may be given as integers or as objects
with a ``data_ptr()`` method (torch tensors); streams as integers, None (the
null stream) or objects with a ``cuda_stream`` attribute.  A negative return
code raises :class:`SweepError` carrying the library's error text.

Importing this module fails loudly when the library has not been built.
"""
import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "libilpsweep.so")

# ---------------------------------------------------------------- constants
OK, EINVAL, EALIGN, EOCCUPANCY, EHIP, ENOMEM, ENODEV = 0, -1, -2, -3, -4, -5, -6
FIXED_WORK, FIXED_ITERS, PER_THREAD_FLOOR = 0, 1, 2
CACHE_DEFAULT, CACHE_NT, CACHE_BYPASS_L1, CACHE_BYPASS_L1_NT = 0, 1, 2, 3
POLICY_NAMES = {"default": 0, "nt": 1, "bypass_l1": 2, "bypass_l1_nt": 3}
KIND_PLAIN, KIND_LDS_ASYNC, KIND_LDS_MATCHED = 0, 1, 2
ORDER_ROUND_ROBIN, ORDER_BLOCKED, ORDER_STRIDED = 0, 1, 2
F32, BF16, FP8_E4M3 = 0, 1, 2


class sweep_wave_rec_t(C.Structure):
    _fields_ = [("sum32", C.c_uint32), ("xor32", C.c_uint32),
                ("hw_id", C.c_uint32), ("xcc_id", C.c_uint32),
                ("t0", C.c_uint64), ("t1", C.c_uint64)]


class sweep_opts_t(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("cache_policy", C.c_int),
                ("mode", C.c_int), ("fixed_iters", C.c_uint32),
                ("grid_wgs", C.c_uint32), ("pin_occupancy", C.c_int),
                ("wave_out", C.c_void_p), ("lane_out", C.c_void_p),
                ("order", C.c_int), ("wave_out_cap", C.c_uint64),
                ("lane_out_cap", C.c_uint64), ("fuse", C.c_int)]


class sweep_result_t(C.Structure):
    _fields_ = [("target_loads", C.c_uint64), ("issued_loads", C.c_uint64),
                ("issued_bytes", C.c_uint64), ("mismatch", C.c_double),
                ("sum32", C.c_uint32), ("xor32", C.c_uint32),
                ("grid_wgs", C.c_uint32), ("wg_threads", C.c_uint32),
                ("waves", C.c_uint32), ("iters_min", C.c_uint32),
                ("iters_max", C.c_uint32), ("max_wgs_per_cu", C.c_uint32),
                ("vgprs", C.c_uint32), ("sgprs", C.c_uint32),
                ("lds_bytes", C.c_uint32), ("scratch_bytes", C.c_uint32),
                ("window_ticks", C.c_uint64), ("window_ns", C.c_double),
                ("event_ms", C.c_double), ("gbps", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class sweep_plan_t(C.Structure):
    _fields_ = [("grid_wgs", C.c_uint32), ("wg_threads", C.c_uint32),
                ("waves", C.c_uint32), ("n_vec", C.c_uint64),
                ("Q", C.c_uint64), ("issued_loads", C.c_uint64),
                ("issued_bytes", C.c_uint64), ("iters_min", C.c_uint32),
                ("iters_max", C.c_uint32), ("mismatch", C.c_double),
                ("lds_pad_bytes", C.c_uint32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class sweep_device_t(C.Structure):
    _fields_ = [("ordinal", C.c_int), ("arch", C.c_char * 64),
                ("num_cus", C.c_uint32), ("lds_per_cu", C.c_uint32),
                ("lds_per_wg_max", C.c_uint32), ("l2_bytes", C.c_uint32),
                ("hbm_bytes", C.c_uint64), ("wall_clock_hz", C.c_double),
                ("calibrated_hz", C.c_double), ("clock_khz", C.c_int),
                ("mem_clock_khz", C.c_int), ("mem_bus_bits", C.c_int)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["arch"] = self.arch.decode()
        return d


class sweep_chase_t(C.Structure):
    _fields_ = [("final_index", C.c_uint32), ("hops", C.c_uint32),
                ("wall_ticks", C.c_uint64), ("ns_per_hop", C.c_double),
                ("shader_clock_hz", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class sweep_walker_t(C.Structure):
    _fields_ = [("final_index", C.c_uint32), ("xcc_id", C.c_uint32),
                ("hops", C.c_uint32), ("reserved", C.c_uint32),
                ("wall_ticks", C.c_uint64), ("ns_per_hop", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class sweep_cell_t(C.Structure):
    _fields_ = [("kind", C.c_int), ("K", C.c_int), ("vec_width", C.c_int),
                ("waves_per_cu", C.c_int), ("cache_policy", C.c_int),
                ("mode", C.c_int), ("fixed_iters", C.c_uint32),
                ("grid_wgs", C.c_uint32), ("buf", C.c_void_p),
                ("bytes", C.c_size_t), ("total_logical_loads", C.c_uint64),
                ("order", C.c_int)]


# symbol -> (restype, argtypes); every function declared in the header
_P = C.c_void_p
_SIG = {
    "sweep_init": (C.c_int, [C.c_int]),
    "sweep_shutdown": (C.c_int, []),
    "sweep_device_info": (C.c_int, [C.POINTER(sweep_device_t)]),
    "sweep_calibrate_clock": (C.c_int, [C.c_double, C.POINTER(C.c_double)]),
    "sweep_plan": (C.c_int, [C.c_size_t, C.c_int, C.c_int, C.c_int, C.c_uint64,
                             C.c_int, C.c_uint32, C.c_uint32, C.c_uint32,
                             C.c_int, C.POINTER(sweep_plan_t)]),
    "sweep_fill_u32": (C.c_int, [_P, C.c_size_t, C.c_uint64, _P]),
    "sweep_plain": (C.c_int, [_P, C.c_size_t, C.c_int, C.c_int, C.c_int,
                              C.c_uint64, C.POINTER(sweep_opts_t),
                              C.POINTER(sweep_result_t)]),
    "sweep_plain_noalloc": (C.c_int, [_P, C.c_size_t, C.c_int, C.c_int, C.c_int,
                                      C.c_uint64, C.POINTER(sweep_opts_t),
                                      C.POINTER(sweep_result_t)]),
    "sweep_lds_async": (C.c_int, [_P, C.c_size_t, C.c_int, C.c_int, C.c_int,
                                  C.c_uint64, C.POINTER(sweep_opts_t),
                                  C.POINTER(sweep_result_t)]),
    "sweep_lds_matched_plain": (C.c_int, [_P, C.c_size_t, C.c_int, C.c_int,
                                          C.c_int, C.c_uint64,
                                          C.POINTER(sweep_opts_t),
                                          C.POINTER(sweep_result_t)]),
    "sweep_two_stream": (C.c_int, [_P, C.c_size_t, C.c_int, C.c_int, C.c_int,
                                   C.c_uint64, C.POINTER(sweep_opts_t),
                                   C.POINTER(sweep_result_t)]),
    "sweep_two_stream_kind": (C.c_int, [_P, C.c_size_t, C.c_int, C.c_int, C.c_int,
                                        C.c_int, C.c_uint64, C.POINTER(sweep_opts_t),
                                        C.POINTER(sweep_result_t)]),
    "sweep_two_stream_split": (C.c_int, [_P, C.c_size_t, C.c_int, C.c_int, C.c_int,
                                         C.c_int, C.c_uint64, C.POINTER(sweep_opts_t),
                                         C.POINTER(sweep_result_t)]),
    "sweep_run": (C.c_int, [C.POINTER(sweep_cell_t), C.c_int,
                            C.POINTER(sweep_opts_t), C.POINTER(sweep_result_t)]),
    "sweep_batched": (C.c_int, [C.POINTER(sweep_cell_t), C.c_int,
                                C.POINTER(sweep_opts_t),
                                C.POINTER(sweep_result_t),
                                C.POINTER(C.c_double)]),
    "sweep_graph_create": (C.c_int, [C.POINTER(sweep_cell_t), C.c_int,
                                     C.POINTER(sweep_opts_t), C.POINTER(_P)]),
    "sweep_graph_launch": (C.c_int, [_P, _P, C.POINTER(sweep_result_t),
                                     C.POINTER(C.c_double)]),
    "sweep_graph_destroy": (C.c_int, [_P]),
    "sweep_autotune": (C.c_int, [_P, C.c_size_t, C.POINTER(C.c_int), C.c_int,
                                 C.POINTER(C.c_int), C.c_int,
                                 C.POINTER(C.c_int), C.c_int, C.c_int, C.c_int,
                                 C.POINTER(sweep_cell_t),
                                 C.POINTER(C.c_double)]),
    "sweep_reduce_fp": (C.c_int, [_P, C.c_size_t, C.c_int, C.c_int,
                                  C.POINTER(sweep_opts_t),
                                  C.POINTER(C.c_double),
                                  C.POINTER(sweep_result_t)]),
    "sweep_chase": (C.c_int, [_P, C.c_size_t, C.c_uint32, C.c_uint32, C.c_uint32,
                              C.c_int, _P, C.c_uint32, _P,
                              C.POINTER(sweep_chase_t)]),
    "sweep_xcd_subset": (C.c_int, [_P, C.c_size_t, C.c_int, C.c_uint32,
                                   C.POINTER(sweep_opts_t), C.POINTER(sweep_result_t)]),
    "sweep_xcd_split": (C.c_int, [_P, C.c_size_t, C.c_int, C.POINTER(C.c_double),
                                  C.POINTER(sweep_opts_t), C.POINTER(sweep_result_t)]),
    "sweep_chase_walkers": (C.c_int, [_P, C.c_size_t, C.POINTER(C.c_uint32), C.c_int,
                                      C.c_uint32, C.c_uint32, C.c_int, _P,
                                      C.POINTER(sweep_walker_t)]),
    "sweep_strerror": (C.c_char_p, [C.c_int]),
    "sweep_last_error": (C.c_char_p, []),
    "sweep_version": (C.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -m paper_2608_15764_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIG.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class SweepError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        text = lib.sweep_last_error().decode() or lib.sweep_strerror(code).decode()
        super().__init__(f"{where}: {lib.sweep_strerror(code).decode()} ({code}): {text}")


def _check(rc, where):
    if rc != OK:
        raise SweepError(rc, where)


def _ptr(x):
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return int(x)


def _stream(s):
    if s is None:
        return None
    if hasattr(s, "cuda_stream"):
        return s.cuda_stream
    return int(s)


def _nbytes(x):
    """Size in bytes of a tensor-like buffer, or None for a raw pointer."""
    if hasattr(x, "numel") and hasattr(x, "element_size"):
        return x.numel() * x.element_size()
    return None


def _cap(buf, cap, item_bytes, name):
    """Capacity in items of an output buffer: from the tensor's size, or the
    caller's ``cap`` for a raw pointer (required then)."""
    if buf is None:
        return 0
    if cap is not None:
        return int(cap)
    n = _nbytes(buf)
    if n is None:
        raise ValueError(f"{name} is a raw pointer: give {name}_cap")
    return n // item_bytes


def make_opts(stream=None, cache_policy=CACHE_DEFAULT, mode=FIXED_WORK,
              fixed_iters=0, grid_wgs=0, pin_occupancy=True, wave_out=None,
              lane_out=None, order=ORDER_ROUND_ROBIN, wave_out_cap=None,
              lane_out_cap=None, fuse=False):
    """Options block.  ``wave_out`` / ``lane_out`` capacities (records of 32
    bytes / lanes of 8 bytes) are taken from the tensors' sizes unless given."""
    o = sweep_opts_t()
    o.stream = _stream(stream)
    o.cache_policy = cache_policy
    o.mode = mode
    o.fixed_iters = fixed_iters
    o.grid_wgs = grid_wgs
    o.pin_occupancy = 1 if pin_occupancy else 0
    o.wave_out = _ptr(wave_out)
    o.lane_out = _ptr(lane_out)
    o.order = order
    o.wave_out_cap = _cap(wave_out, wave_out_cap, C.sizeof(sweep_wave_rec_t), "wave_out")
    o.lane_out_cap = _cap(lane_out, lane_out_cap, 8, "lane_out")
    o.fuse = 1 if fuse else 0
    return o


# ------------------------------------------------------------ entry points
def sweep_init(ordinal=0):
    """Initialise the library on HIP device ``ordinal`` (makes it current)."""
    _check(lib.sweep_init(ordinal), "sweep_init")


def sweep_shutdown():
    """Free the library's device memory and events on every device."""
    _check(lib.sweep_shutdown(), "sweep_shutdown")


def sweep_device_info():
    """Properties of the current device as a dict (CUs, LDS, caches, clocks)."""
    d = sweep_device_t()
    _check(lib.sweep_device_info(C.byref(d)), "sweep_device_info")
    return d.as_dict()


def sweep_calibrate_clock(seconds=0.2):
    """Measure the device wall clock against the host over about ``seconds``; returns Hz."""
    hz = C.c_double()
    _check(lib.sweep_calibrate_clock(seconds, C.byref(hz)), "sweep_calibrate_clock")
    return hz.value


def sweep_plan(bytes_, K, vec_width, waves_per_cu, total_logical_loads,
               mode=FIXED_WORK, fixed_iters=0, num_cus=256, grid_wgs=0,
               order=ORDER_ROUND_ROBIN):
    """Host-only fixed-work plan of a cell (no GPU needed); returns a dict."""
    p = sweep_plan_t()
    _check(lib.sweep_plan(bytes_, K, vec_width, waves_per_cu,
                          total_logical_loads, mode, fixed_iters, num_cus,
                          grid_wgs, order, C.byref(p)), "sweep_plan")
    return p.as_dict()


def sweep_fill_u32(buf, bytes_, seed, stream=None):
    """Fill ``bytes_`` of ``buf`` with the seeded SplitMix64 words (untimed setup)."""
    _check(lib.sweep_fill_u32(_ptr(buf), bytes_, seed & (2**64 - 1),
                              _stream(stream)), "sweep_fill_u32")


def _cell_call(fn, name, buf, bytes_, K, vec_width, waves_per_cu, L, opts):
    r = sweep_result_t()
    o = opts if opts is not None else make_opts()
    _check(fn(_ptr(buf), bytes_, K, vec_width, waves_per_cu, L, C.byref(o),
              C.byref(r)), name)
    return r.as_dict()


def sweep_plain(buf, bytes_, K, vec_width, waves_per_cu, total_logical_loads,
                opts=None):
    """One plain K-load cell; returns the result dict (sinks, issued loads, window, GB/s)."""
    return _cell_call(lib.sweep_plain, "sweep_plain", buf, bytes_, K,
                      vec_width, waves_per_cu, total_logical_loads, opts)


def sweep_plain_noalloc(buf, bytes_, K, vec_width, waves_per_cu, total_logical_loads,
                        opts=None):
    """``sweep_plain`` with no allocation: its scratch is a static device array."""
    return _cell_call(lib.sweep_plain_noalloc, "sweep_plain_noalloc", buf, bytes_, K,
                      vec_width, waves_per_cu, total_logical_loads, opts)


def sweep_lds_async(buf, bytes_, depth, vec_width, waves_per_cu,
                    total_logical_loads, opts=None):
    """One LDS-direct ring cell of depth ``depth`` (16-byte requests)."""
    return _cell_call(lib.sweep_lds_async, "sweep_lds_async", buf, bytes_,
                      depth, vec_width, waves_per_cu, total_logical_loads, opts)


def sweep_lds_matched_plain(buf, bytes_, depth, vec_width, waves_per_cu,
                            total_logical_loads, opts=None):
    """The matched register ring of ``sweep_lds_async`` (load, LDS write, LDS read)."""
    return _cell_call(lib.sweep_lds_matched_plain, "sweep_lds_matched_plain",
                      buf, bytes_, depth, vec_width, waves_per_cu,
                      total_logical_loads, opts)


def sweep_two_stream(buf, bytes_, depth, waves_plain, waves_async,
                     total_logical_loads, opts=None):
    """Two co-resident streams in one workgroup, plain and LDS-direct; two result dicts."""
    r = (sweep_result_t * 2)()
    o = opts if opts is not None else make_opts()
    _check(lib.sweep_two_stream(_ptr(buf), bytes_, depth, waves_plain,
                                waves_async, total_logical_loads, C.byref(o),
                                r), "sweep_two_stream")
    return r[0].as_dict(), r[1].as_dict()


def sweep_two_stream_kind(buf, bytes_, depth, waves_a, waves_b, kind_b,
                          total_logical_loads, opts=None):
    """Two co-resident streams in one workgroup, stream B of ``kind_b``; two result dicts."""
    r = (sweep_result_t * 2)()
    o = opts if opts is not None else make_opts()
    _check(lib.sweep_two_stream_kind(_ptr(buf), bytes_, depth, waves_a, waves_b,
                                     kind_b, total_logical_loads, C.byref(o), r),
           "sweep_two_stream_kind")
    return r[0].as_dict(), r[1].as_dict()


def sweep_two_stream_split(buf, bytes_, depth, waves_a, waves_b, kind_b,
                           total_logical_loads, opts=None):
    """The two streams on different CUs; two result dicts."""
    r = (sweep_result_t * 2)()
    o = opts if opts is not None else make_opts()
    _check(lib.sweep_two_stream_split(_ptr(buf), bytes_, depth, waves_a, waves_b,
                                      kind_b, total_logical_loads, C.byref(o), r),
           "sweep_two_stream_split")
    return r[0].as_dict(), r[1].as_dict()


def make_cell(buf, bytes_, K, vec_width, waves_per_cu, total_logical_loads,
              kind=KIND_PLAIN, cache_policy=CACHE_DEFAULT, mode=FIXED_WORK,
              fixed_iters=0, grid_wgs=0, order=ORDER_ROUND_ROBIN):
    """A ``sweep_cell_t`` for the sweep driver, graphs and the batched sweep."""
    c = sweep_cell_t()
    c.kind = kind
    c.K = K
    c.vec_width = vec_width
    c.waves_per_cu = waves_per_cu
    c.cache_policy = cache_policy
    c.mode = mode
    c.fixed_iters = fixed_iters
    c.grid_wgs = grid_wgs
    c.buf = _ptr(buf)
    c.bytes = bytes_
    c.total_logical_loads = total_logical_loads
    c.order = order
    return c


def cell_array(cells):
    """A ctypes array of cells (build once, pass to sweep_run repeatedly)."""
    if isinstance(cells, C.Array):
        return cells
    arr = (sweep_cell_t * len(cells))()
    for i, c in enumerate(cells):
        arr[i] = c if isinstance(c, sweep_cell_t) else make_cell(**c)
    return arr


def result_dicts(raw):
    """Convert a ctypes result array into a list of dicts."""
    return [r.as_dict() for r in raw]


def sweep_run(cells, opts=None, raw=False):
    """Run cells back to back.  ``raw=True`` returns the ctypes result array
    (convert with :func:`result_dicts`), keeping conversion out of timing."""
    arr = cell_array(cells)
    res = (sweep_result_t * len(arr))()
    o = opts if opts is not None else make_opts()
    _check(lib.sweep_run(arr, len(arr), C.byref(o), res), "sweep_run")
    return res if raw else result_dicts(res)


def sweep_batched(cells, opts=None, raw=False):
    """Capture ``cells`` into a hipGraph, launch it once, destroy it; (results, graph ms)."""
    arr = cell_array(cells)
    res = (sweep_result_t * len(arr))()
    o = opts if opts is not None else make_opts()
    ms = C.c_double()
    _check(lib.sweep_batched(arr, len(arr), C.byref(o), res, C.byref(ms)),
           "sweep_batched")
    return (res if raw else result_dicts(res)), ms.value


class SweepGraph:
    """Handle of a captured sweep: the C handle and its cell count.  Usable
    as a context manager that destroys the graph on exit."""

    def __init__(self, handle, n):
        self.handle = handle
        self.n = n

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        sweep_graph_destroy(self)
        return False


def sweep_graph_create(cells, opts=None):
    """Capture ``cells`` once into a replayable graph (a context manager)."""
    arr = cell_array(cells)
    h = _P()
    o = opts if opts is not None else make_opts()
    _check(lib.sweep_graph_create(arr, len(arr), C.byref(o), C.byref(h)),
           "sweep_graph_create")
    return SweepGraph(h.value, len(arr))


def sweep_graph_launch(graph, stream=None, raw=False):
    """Replay a captured graph; (results, graph ms), or raw ctypes results."""
    res = (sweep_result_t * graph.n)()
    ms = C.c_double()
    _check(lib.sweep_graph_launch(graph.handle, _stream(stream), res,
                                  C.byref(ms)), "sweep_graph_launch")
    return (res if raw else result_dicts(res)), ms.value


def sweep_graph_destroy(graph):
    """Free a captured graph and its scratch."""
    if graph is not None and graph.handle:
        _check(lib.sweep_graph_destroy(graph.handle), "sweep_graph_destroy")
        graph.handle = None


def sweep_autotune(buf, bytes_, vec_widths, Ks, waves_per_cu,
                   cache_policy=CACHE_DEFAULT, reps=3):
    """Time every (width, K, waves) candidate of a plain cell; the best and its GB/s."""
    vw = (C.c_int * len(vec_widths))(*vec_widths)
    ks = (C.c_int * len(Ks))(*Ks)
    ws = (C.c_int * len(waves_per_cu))(*waves_per_cu)
    best = sweep_cell_t()
    g = C.c_double()
    _check(lib.sweep_autotune(_ptr(buf), bytes_, vw, len(vw), ks, len(ks), ws,
                              len(ws), cache_policy, reps, C.byref(best),
                              C.byref(g)), "sweep_autotune")
    return {"K": best.K, "vec_width": best.vec_width,
            "waves_per_cu": best.waves_per_cu,
            "cache_policy": best.cache_policy}, g.value


def sweep_reduce_fp(payload, n_elems, dtype, waves_per_cu=32, opts=None):
    """The compensated streaming sum of an FP32/BF16/FP8 payload; (FP64 sum, result dict)."""
    s = C.c_double()
    r = sweep_result_t()
    o = opts if opts is not None else make_opts()
    _check(lib.sweep_reduce_fp(_ptr(payload), n_elems, dtype, waves_per_cu,
                               C.byref(o), C.byref(s), C.byref(r)),
           "sweep_reduce_fp")
    return s.value, r.as_dict()


def sweep_chase(chain, bytes_, start, warm_hops, hops, cache_policy=CACHE_DEFAULT,
                samples=None, n_samples=0, stream=None):
    """The dependent pointer chase of one lane; a result dict (final index, ns per hop)."""
    o = sweep_chase_t()
    _check(lib.sweep_chase(_ptr(chain), bytes_, start, warm_hops, hops,
                           cache_policy, _ptr(samples), n_samples,
                           _stream(stream), C.byref(o)), "sweep_chase")
    return o.as_dict()


def sweep_xcd_subset(buf, bytes_, waves_per_cu, xcd_mask, opts=None):
    """The plain K = 8 read run only by the workgroups of the XCDs in
    ``xcd_mask`` (bit x: XCD x); returns the result dict of one launch."""
    r = sweep_result_t()
    o = opts if opts is not None else make_opts()
    _check(lib.sweep_xcd_subset(_ptr(buf), bytes_, waves_per_cu, xcd_mask, C.byref(o),
                                C.byref(r)), "sweep_xcd_subset")
    return r.as_dict()


def sweep_xcd_split(buf, bytes_, waves_per_cu, weights, opts=None):
    """The same read with a contiguous share of the groups per XCD, in
    proportion to ``weights`` (8 values, XCD 0 first)."""
    if len(weights) != 8:
        raise ValueError("weights takes one value per XCD (8)")
    w = (C.c_double * 8)(*[float(v) for v in weights])
    r = sweep_result_t()
    o = opts if opts is not None else make_opts()
    _check(lib.sweep_xcd_split(_ptr(buf), bytes_, waves_per_cu, w, C.byref(o), C.byref(r)),
           "sweep_xcd_split")
    return r.as_dict()


MAX_WALKERS = 64


def sweep_chase_walkers(chain, bytes_, starts, warm_hops, hops, cache_policy=CACHE_DEFAULT,
                        stream=None):
    """One dependent-chain walker per start index, all at once; returns one
    dict per walker (final index, the XCD it ran on, ns per hop)."""
    n = len(starts)
    st = (C.c_uint32 * max(n, 1))(*[int(v) for v in starts])
    out = (sweep_walker_t * max(n, 1))()
    _check(lib.sweep_chase_walkers(_ptr(chain), bytes_, st, n, warm_hops, hops,
                                   cache_policy, _stream(stream), out),
           "sweep_chase_walkers")
    return [out[i].as_dict() for i in range(n)]


def sweep_strerror(code):
    """Text of an error code."""
    return lib.sweep_strerror(code).decode()


def sweep_last_error():
    """Text of the calling thread's last error."""
    return lib.sweep_last_error().decode()


def sweep_version():
    """Library version string."""
    return lib.sweep_version().decode()
