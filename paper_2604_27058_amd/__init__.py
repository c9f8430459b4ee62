"""MI355X (gfx950) sample-many engine for near-Clifford circuits.

Thin ctypes binding over libclifft.so (declared in include/clifft.h): the
functions keep the C names; this module only marshals arguments.  All
compilation runs in the library's host compiler and all sampling runs in its
HIP kernels; PyTorch only provides device memory and streams.  If the
library is missing this module raises instead of falling back to anything.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libclifft.so")

CLIFFT_FP32, CLIFFT_FP64 = 0, 1
STATUS = {0: "OK", 1: "E_PARSE", 2: "E_UNSUPPORTED", 3: "E_CAPACITY", 4: "E_INVALID_ARG", 5: "E_DEVICE",
          6: "E_IMPOSSIBLE_OUTCOME"}


class ClifftError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class clifft_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "num_qubits", "frame_words", "k_max", "num_events", "num_measurements", "num_detectors",
        "num_observables", "num_noise_sites", "num_instructions", "num_random_events", "num_active_events",
        "num_probes", "num_postselected")]


class clifft_cost(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "int_ops", "flops", "vector_bytes", "record_bytes", "expected_faults", "instructions",
        "int_ops_bitsliced", "vector_bytes_fused", "vector_bytes_fused_group", "vector_bytes_fused_batch",
        "paired_measurements")]


class clifft_compile_opts(ctypes.Structure):
    _fields_ = [("hir_passes", ctypes.c_int32), ("k_limit", ctypes.c_int32), ("drop_phases", ctypes.c_int32),
                ("postselect", ctypes.POINTER(ctypes.c_uint64)), ("postselect_words", ctypes.c_int32)]


class clifft_launch(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("threads_per_shot", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("vector_in_hbm", ctypes.c_int32), ("specialize", ctypes.c_int32), ("split", ctypes.c_int32)]


_lib = None


def lib():
    """Load libclifft.so (built in-tree by build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libclifft.so is not built (run paper_2604_27058_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, sz, i32p = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int32)
        L.clifft_compile.argtypes = [ctypes.c_char_p, sz, ctypes.POINTER(clifft_compile_opts), ctypes.POINTER(vp)]
        L.clifft_program_info.argtypes = [vp, ctypes.POINTER(clifft_info)]
        L.clifft_k_profile.argtypes = [vp, i32p, sz, ctypes.POINTER(sz)]
        L.clifft_event_classes.argtypes = [vp, i32p, sz, ctypes.POINTER(sz)]
        L.clifft_pair_orders.argtypes = [vp, i32p, sz, ctypes.POINTER(sz)]
        L.clifft_final_slots.argtypes = [vp, i32p, i32p]
        L.clifft_workspace_size.argtypes = [vp, ctypes.POINTER(clifft_launch), u64, ctypes.POINTER(sz)]
        L.clifft_sample.argtypes = [vp, u64, u64, u64, ctypes.POINTER(clifft_launch), vp, sz, vp, vp, vp, vp]
        L.clifft_sample_noalloc.argtypes = [vp, u64, u64, u64, ctypes.POINTER(clifft_launch), vp, vp, vp, vp]
        L.clifft_sample_expval.argtypes = [vp, u64, u64, u64, ctypes.POINTER(clifft_launch), vp, sz, vp, vp, vp, vp,
                                           vp]
        L.clifft_sample_trace.argtypes = [vp, u64, u64, u64, ctypes.POINTER(clifft_launch), vp, vp, vp, vp, vp, vp,
                                          sz, vp, vp, vp, vp]
        L.clifft_sample_stratified.argtypes = [vp, u64, u64, u64, ctypes.c_int32, ctypes.POINTER(clifft_launch), vp,
                                               sz, vp, vp, vp, vp]
        L.clifft_fault_count_pmf.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        L.clifft_cost_model.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(clifft_cost)]
        L.clifft_resolve_launch.argtypes = [vp, ctypes.POINTER(clifft_launch), u64, ctypes.POINTER(clifft_launch)]
        L.clifft_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(u64), ctypes.POINTER(u64),
                                          ctypes.POINTER(clifft_launch), ctypes.POINTER(vp)]
        L.clifft_batch_sizes.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64),
                                         ctypes.POINTER(sz), i32p]
        L.clifft_batch_layout.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(u64), ctypes.POINTER(u64),
                                          ctypes.POINTER(u64)]
        L.clifft_batch_sample.argtypes = [vp, vp, sz, vp, vp, vp, vp]
        L.clifft_batch_free.argtypes = [vp]
        L.clifft_autotune.argtypes = [vp, u64, ctypes.c_int32, vp, ctypes.POINTER(clifft_launch)]
        L.clifft_specialize.argtypes = [vp, ctypes.c_char_p, sz]
        L.clifft_program_free.argtypes = [vp]
        L.clifft_probe.argtypes = [ctypes.c_int32, vp, vp, u64, ctypes.c_int32, vp]
        L.clifft_last_error.restype = ctypes.c_char_p
        for f in ("clifft_compile", "clifft_program_info", "clifft_k_profile", "clifft_event_classes",
                  "clifft_final_slots", "clifft_workspace_size", "clifft_sample", "clifft_sample_noalloc",
                  "clifft_sample_expval", "clifft_sample_stratified", "clifft_fault_count_pmf",
                  "clifft_sample_trace",
                  "clifft_cost_model", "clifft_resolve_launch", "clifft_batch_create", "clifft_batch_sizes",
                  "clifft_batch_layout", "clifft_batch_sample", "clifft_autotune", "clifft_specialize",
                  "clifft_probe"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        raise ClifftError(st, lib().clifft_last_error().decode())


def probe(kind, dst, src=None, n=0, grid=1, stream=None):
    """clifft_probe on device tensors (kind 0: copy n bytes src -> dst;
    kind 1: n iterations of 16 VALU instructions per thread into dst)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().clifft_probe(kind, dst.data_ptr(), None if src is None else src.data_ptr(), n, grid, s.cuda_stream))


def make_launch(precision="f32", threads_per_shot=0, grid=0, vector_in_hbm=0, specialize=0, split=0):
    p = CLIFFT_FP64 if precision in ("f64", CLIFFT_FP64) else CLIFFT_FP32
    return clifft_launch(p, threads_per_shot, grid, vector_in_hbm, specialize, split)


class Program:
    """A compiled circuit (clifft_compile; keyword options as in
    clifft_compile_opts; postselect: None, "all" or detector indices)."""

    def __init__(self, text, hir_passes=0, k_limit=0, drop_phases=0, postselect=None):
        h = ctypes.c_void_p()
        b = text.encode()
        opts = clifft_compile_opts(hir_passes, k_limit, drop_phases)
        mask = None
        if isinstance(postselect, str):
            if postselect != "all":
                raise ValueError("postselect: 'all' or detector indices")
            opts.postselect_words = -1  # every detector
        elif postselect is not None:
            idx = [int(d) for d in postselect]
            if any(d < 0 for d in idx):
                raise ValueError("postselect: negative detector index")
            words = max((max(idx, default=-1) + 64) // 64, 1)
            mask = (ctypes.c_uint64 * words)()
            for d in idx:
                mask[d // 64] |= 1 << (d % 64)
            opts.postselect = ctypes.cast(mask, ctypes.POINTER(ctypes.c_uint64))
            opts.postselect_words = words
        _check(lib().clifft_compile(b, len(b), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        inf = clifft_info()
        _check(lib().clifft_program_info(h, ctypes.byref(inf)))
        self.info = {f: getattr(inf, f) for f, _ in clifft_info._fields_}
        for f, _ in clifft_info._fields_:
            setattr(self, f, getattr(inf, f))
        if postselect is None:
            self.postselected = []
        elif isinstance(postselect, str):
            self.postselected = list(range(self.num_detectors))
        else:
            self.postselected = sorted(set(int(d) for d in postselect))

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.clifft_program_free(self._h)
            self._h = None

    def _arr(self, fn):
        n = ctypes.c_size_t()
        _check(fn(self._h, None, 0, ctypes.byref(n)))
        out = (ctypes.c_int32 * max(n.value, 1))()
        _check(fn(self._h, out, n.value, ctypes.byref(n)))
        return list(out)[: n.value]

    def k_profile(self):
        return self._arr(lib().clifft_k_profile)

    def event_classes(self):
        return self._arr(lib().clifft_event_classes)

    def pair_orders(self):
        """The compiler's paired-pass item orders (clifft_pair_orders): a
        list of dicts (instr, kind, n, and per element size f32/f64: nv,
        pos, v)."""
        a = self._arr(lib().clifft_pair_orders)
        out = []
        for i in range(0, len(a), 25):
            e = dict(instr=a[i], kind=a[i + 1], n=a[i + 2])
            for j, prec in enumerate(("f32", "f64")):
                b = i + 3 + 11 * j
                e[prec] = dict(nv=a[b], pos=a[b + 2: b + 2 + a[b + 1]], v=[x & 0xFFFFFFFF for x in a[b + 7: b + 11]][: a[b]])
            out.append(e)
        return out

    def final_slots(self):
        out = (ctypes.c_int32 * max(self.k_max, 1))()
        k = ctypes.c_int32()
        _check(lib().clifft_final_slots(self._h, out, ctypes.byref(k)))
        return list(out)[: k.value]

    def cost_model(self, precision="f32"):
        """Per-shot algorithmic work (clifft_cost_model) as a dict."""
        c = clifft_cost()
        _check(lib().clifft_cost_model(self._h, CLIFFT_FP64 if precision == "f64" else CLIFFT_FP32,
                                       ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in clifft_cost._fields_}

    def resolve_launch(self, shots, launch=None):
        """The configuration clifft_sample would use (dict)."""
        out = clifft_launch()
        _check(lib().clifft_resolve_launch(self._h, None if launch is None else ctypes.byref(launch), shots,
                                           ctypes.byref(out)))
        return {f: getattr(out, f) for f, _ in clifft_launch._fields_}

    def specialize(self):
        """clifft_specialize: build the program-specialized bit-sliced kernel
        (host only); returns the library's note (reason or compiler log)."""
        buf = ctypes.create_string_buffer(4096)
        _check(lib().clifft_specialize(self._h, buf, len(buf)))
        return buf.value.decode(errors="replace")

    def autotune(self, shots, precision="f32"):
        """clifft_autotune: time the launch shapes, keep the fastest (dict)."""
        import torch
        out = clifft_launch()
        _check(lib().clifft_autotune(self._h, shots, CLIFFT_FP64 if precision == "f64" else CLIFFT_FP32,
                                     torch.cuda.current_stream().cuda_stream, ctypes.byref(out)))
        return {f: getattr(out, f) for f, _ in clifft_launch._fields_}

    def workspace_size(self, launch=None, shots=1 << 20):
        n = ctypes.c_size_t()
        _check(lib().clifft_workspace_size(self._h, None if launch is None else ctypes.byref(launch), shots,
                                           ctypes.byref(n)))
        return n.value

    # ---- sampling through torch-owned device buffers
    def alloc_outputs(self, shots, device="cuda"):
        import torch
        words = (shots + 63) // 64
        mk = lambda rows: torch.empty((rows, words), dtype=torch.int64, device=device)
        return mk(self.num_measurements), mk(self.num_detectors), mk(self.num_observables)

    def alloc_workspace(self, launch=None, device="cuda", shots=1 << 20):
        import torch
        n = self.workspace_size(launch, shots)
        return torch.empty(max(n, 1), dtype=torch.uint8, device=device) if n else None

    def sample(self, shots, seed=0, offset=0, launch=None, outputs=None, workspace=None, stream=None):
        """Queue clifft_sample on the current stream; returns (meas, det, obs)
        int64 device tensors holding the bit-packed uint64 record words."""
        import torch
        meas, det, obs = outputs if outputs is not None else self.alloc_outputs(shots)
        if workspace is None:
            workspace = self.alloc_workspace(launch, shots=shots)
        s = stream if stream is not None else torch.cuda.current_stream()
        ptr = lambda t: t.data_ptr() if (t is not None and t.numel()) else None
        _check(lib().clifft_sample(self._h, shots, seed, offset, None if launch is None else ctypes.byref(launch),
                                   ptr(workspace), 0 if workspace is None else workspace.numel(), ptr(meas),
                                   ptr(det), ptr(obs), s.cuda_stream))
        return meas, det, obs

    def sample_expval(self, shots, seed=0, offset=0, launch=None, outputs=None, workspace=None, stream=None):
        """clifft_sample_expval: records as in sample() and the probes'
        values, a [num_probes, shots] float64 device tensor."""
        import torch
        meas, det, obs = outputs if outputs is not None else self.alloc_outputs(shots)
        if workspace is None:
            workspace = self.alloc_workspace(launch, shots=shots)
        ev = torch.zeros((max(self.num_probes, 1), shots), dtype=torch.float64, device="cuda")
        s = stream if stream is not None else torch.cuda.current_stream()
        ptr = lambda t: t.data_ptr() if (t is not None and t.numel()) else None
        _check(lib().clifft_sample_expval(self._h, shots, seed, offset,
                                          None if launch is None else ctypes.byref(launch), ptr(workspace),
                                          0 if workspace is None else workspace.numel(), ptr(meas), ptr(det),
                                          ptr(obs), ptr(ev), s.cuda_stream))
        return (meas, det, obs), ev[: self.num_probes]

    def sample_stratified(self, shots, faults, seed=0, offset=0, launch=None, outputs=None, workspace=None,
                          stream=None):
        """clifft_sample_stratified: every shot with exactly `faults` faults;
        returns (meas, det, obs) as sample() does."""
        import torch
        meas, det, obs = outputs if outputs is not None else self.alloc_outputs(shots)
        if workspace is None:
            workspace = self.alloc_workspace(launch, shots=shots)
        s = stream if stream is not None else torch.cuda.current_stream()
        ptr = lambda t: t.data_ptr() if (t is not None and t.numel()) else None
        _check(lib().clifft_sample_stratified(self._h, shots, seed, offset, faults,
                                              None if launch is None else ctypes.byref(launch), ptr(workspace),
                                              0 if workspace is None else workspace.numel(), ptr(meas), ptr(det),
                                              ptr(obs), s.cuda_stream))
        return meas, det, obs

    def fault_count_pmf(self, rmax):
        """clifft_fault_count_pmf: P(exactly r faults), r = 0 .. rmax (list)."""
        out = (ctypes.c_double * (rmax + 1))()
        _check(lib().clifft_fault_count_pmf(self._h, rmax, out))
        return list(out)

    def kept(self, det):
        """Kept-shot mask words (int64 tensor, one row) from the detector
        rows of a post-selected program: a shot is kept iff all its
        post-selected detectors read 0."""
        import torch
        keep = torch.full((det.shape[1],), -1, dtype=torch.int64, device=det.device)
        for d in self.postselected:
            keep &= ~det[d]
        return keep

    def sample_noalloc(self, shots, seed=0, offset=0, launch=None, outputs=None, stream=None):
        """Queue clifft_sample_noalloc (no workspace argument; the library's
        fixed device scratch serves the HBM tiers) into `outputs` on the
        current stream; returns (meas, det, obs)."""
        import torch
        meas, det, obs = outputs if outputs is not None else self.alloc_outputs(shots)
        s = stream if stream is not None else torch.cuda.current_stream()
        ptr = lambda t: t.data_ptr() if (t is not None and t.numel()) else None
        _check(lib().clifft_sample_noalloc(self._h, shots, seed, offset,
                                           None if launch is None else ctypes.byref(launch), ptr(meas), ptr(det),
                                           ptr(obs), s.cuda_stream))
        return meas, det, obs

    def sample_trace(self, shots, seed=0, offset=0, launch=None, forced_m=None, forced_faults=None, want_phi=True):
        """Trace mode (testing).  Returns dict of device tensors: meas, det,
        obs, probs [shots, events], phi [shots, 2^k_max] complex128 (None
        when want_phi is false), gamma [shots] complex128."""
        import torch
        meas, det, obs = self.alloc_outputs(shots)
        probs = torch.zeros((shots, max(self.num_events, 1)), dtype=torch.float64, device="cuda")
        phi = torch.zeros((shots, 1 << self.k_max, 2), dtype=torch.float64, device="cuda") if want_phi else None
        gamma = torch.zeros((shots, 2), dtype=torch.float64, device="cuda")
        ws = self.alloc_workspace(launch, shots=shots)
        fm = None if forced_m is None else forced_m.to(device="cuda", dtype=torch.int32).contiguous()
        ff = None if forced_faults is None else forced_faults.to(device="cuda", dtype=torch.int32).contiguous()
        ptr = lambda t: t.data_ptr() if (t is not None and t.numel()) else None
        s = torch.cuda.current_stream()
        _check(lib().clifft_sample_trace(self._h, shots, seed, offset,
                                         None if launch is None else ctypes.byref(launch), ptr(fm), ptr(ff),
                                         ptr(probs), ptr(phi), ptr(gamma), ptr(ws), 0 if ws is None else ws.numel(),
                                         ptr(meas), ptr(det), ptr(obs), s.cuda_stream))
        return dict(meas=meas, det=det, obs=obs, probs=probs[:, : self.num_events],
                    phi=None if phi is None else torch.view_as_complex(phi), gamma=torch.view_as_complex(gamma))


class Batch:
    """Many programs sampled by one persistent launch (clifft_batch_*)."""

    def __init__(self, programs, shots, seeds, precision="f32", threads_per_shot=0, grid=0):
        n = len(programs)
        self.programs = list(programs)  # keep the programs alive
        hs = (ctypes.c_void_p * n)(*[p._h.value for p in programs])
        sh = (ctypes.c_uint64 * n)(*shots)
        sd = (ctypes.c_uint64 * n)(*seeds)
        cfg = make_launch(precision, threads_per_shot=threads_per_shot, grid=grid)
        h = ctypes.c_void_p()
        _check(lib().clifft_batch_create(hs, n, sh, sd, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.shots = list(shots)
        mw, dw, ow, ws = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_size_t()
        tps = (ctypes.c_int32 * n)()
        _check(lib().clifft_batch_sizes(h, ctypes.byref(mw), ctypes.byref(dw), ctypes.byref(ow), ctypes.byref(ws),
                                        tps))
        self.meas_words, self.det_words, self.obs_words = mw.value, dw.value, ow.value
        self.workspace_bytes = ws.value
        self.threads_per_shot = list(tps)
        self.layout = []
        for i in range(n):
            a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
            _check(lib().clifft_batch_layout(h, i, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
            self.layout.append((a.value, b.value, c.value))

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.clifft_batch_free(self._h)
            self._h = None

    def alloc(self, device="cuda"):
        import torch
        mk = lambda n: torch.empty(max(n, 1), dtype=torch.int64, device=device)
        ws = torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=device)
        return (mk(self.meas_words), mk(self.det_words), mk(self.obs_words)), ws

    def sample(self, outputs=None, workspace=None, stream=None):
        import torch
        if outputs is None or workspace is None:
            outputs, workspace = self.alloc()
        s = stream if stream is not None else torch.cuda.current_stream()
        m, d, o = outputs
        _check(lib().clifft_batch_sample(self._h, workspace.data_ptr(), workspace.numel(), m.data_ptr(),
                                         d.data_ptr(), o.data_ptr(), s.cuda_stream))
        return outputs

    def records(self, outputs, i):
        """Program i's (meas, det, obs) rows as [rows, words] views."""
        p = self.programs[i]
        words = (self.shots[i] + 63) // 64
        mo, do, oo = self.layout[i]
        m, d, o = outputs
        return (m[mo: mo + p.num_measurements * words].view(p.num_measurements, words),
                d[do: do + p.num_detectors * words].view(p.num_detectors, words),
                o[oo: oo + p.num_observables * words].view(p.num_observables, words))
