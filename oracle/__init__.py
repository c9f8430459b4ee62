"""Plain FP64 CPU oracle (ctypes wrapper around oracle.c).

TEST INFRASTRUCTURE ONLY: used by tests/, by the smoke check and by the
benchmark's cpu_baseline leg.  The product path never imports this package.
It shares no code with the HIP path.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile oracle.c with gcc (plain C11, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", _SO + ".tmp", os.path.join(_HERE, "oracle.c"), "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
        L.oracle_compile.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(vp), ctypes.c_char_p, i32]
        L.oracle_compile.restype = i32
        L.oracle_free.argtypes = [vp]
        L.oracle_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.oracle_event_classes.argtypes = [vp, ctypes.POINTER(i32)]
        L.oracle_ops.argtypes = [vp, ctypes.POINTER(i32)]
        L.oracle_uclog.argtypes = [vp, ctypes.POINTER(i32), i32]
        L.oracle_uclog.restype = i32
        L.oracle_philox.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.oracle_survival.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
        L.oracle_survival.restype = i32
        L.oracle_faults.argtypes = [vp, u64, u64, ctypes.POINTER(i32)]
        L.oracle_gap_next.argtypes = [ctypes.POINTER(ctypes.c_double), i32, i32, ctypes.c_double]
        L.oracle_gap_next.restype = i32
        L.oracle_trace.argtypes = [vp, u64, u64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_trace.restype = i32
        L.oracle_sample.argtypes = [vp, u64, u64, u64, i32, vp, vp, vp, vp, i32]
        L.oracle_sample.restype = i32
        L.oracle_fault_pmf.argtypes = [vp, i32, vp]
        L.oracle_fault_pmf.restype = i32
        L.oracle_faults_strat.argtypes = [vp, i32, u64, u64, vp]
        L.oracle_faults_strat.restype = i32
        L.oracle_strat_survival.argtypes = [vp, i32, i32, i32]
        L.oracle_strat_survival.restype = ctypes.c_double
        L.oracle_set_postselect.argtypes = [vp, vp, i32]
        L.oracle_set_postselect.restype = i32
        _lib = L
    return _lib


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox(c, k, o)
    return list(o)


def gap_next(S, cur, u):
    S = np.ascontiguousarray(S, dtype=np.float64)
    return lib().oracle_gap_next(S.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(S) - 1, cur, u)


OP_NAMES = ["VCX", "VCZ", "VS", "VH", "EXPAND", "ROT", "PHASE", "MSTATIC", "MRANDOM", "MACTIVE_Z",
            "MACTIVE_X", "CPAULI", "NOISE", "DET", "OBS", "CFEED", "EXPVAL"]


class OracleError(RuntimeError):
    pass


class Program:
    """A circuit compiled by the oracle (the Stim-like text subset its parser accepts)."""

    def __init__(self, text, postselect=None):
        """postselect: None, "all", or an iterable of detector indices whose
        reading 1 rejects the shot (Section 3.2, post-selection)."""
        L = lib()
        h = ctypes.c_void_p()
        err = ctypes.create_string_buffer(512)
        b = text.encode()
        rc = L.oracle_compile(b, len(b), ctypes.byref(h), err, 512)
        if rc != 0:
            raise OracleError(err.value.decode())
        self._h = h
        info = (ctypes.c_int64 * 10)()
        L.oracle_info(h, info)
        (self.nq, self.kmax, self.nevents, self.nrec, self.ndet, self.nobs, self.nsites, self.nops,
         self.nchunks, self.nprobes) = [int(v) for v in info]
        if postselect is not None:
            idx = range(self.ndet) if isinstance(postselect, str) and postselect == "all" else list(postselect)
            mask = np.zeros(max((self.ndet + 63) // 64, 1), np.uint64)
            for d in idx:
                if not 0 <= d < self.ndet:
                    raise OracleError("post-selected detector %d out of range" % d)
                mask[d // 64] |= np.uint64(1) << np.uint64(d % 64)
            if L.oracle_set_postselect(h, mask.ctypes.data, len(mask)) != 0:
                raise OracleError("bad post-selection mask")

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.oracle_free(self._h)
            self._h = None

    def event_classes(self):
        out = np.zeros(max(self.nevents, 1), dtype=np.int32)
        lib().oracle_event_classes(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        return out[: self.nevents]

    def ops(self):
        out = np.zeros((max(self.nops, 1), 4), dtype=np.int32)
        lib().oracle_ops(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        return out[: self.nops]

    def k_profile(self):
        return self.ops()[:, 3]

    def uclog(self):
        n = lib().oracle_uclog(self._h, None, 0)
        out = np.zeros(max(n, 1), dtype=np.int32)
        lib().oracle_uclog(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), n)
        return out[:n].reshape(-1, 4)

    def survival(self, chunk):
        out = np.zeros(4097, dtype=np.float64)
        n = lib().oracle_survival(self._h, chunk, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return out[: n + 1]

    def faults(self, seed, shot):
        out = np.zeros(max(self.nsites, 1), dtype=np.int32)
        lib().oracle_faults(self._h, seed, shot, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        return out[: self.nsites]

    def fault_pmf(self, rmax):
        """P(exactly r noise sites fire), r = 0 .. rmax (Poisson-binomial)."""
        out = np.zeros(rmax + 1)
        if lib().oracle_fault_pmf(self._h, rmax, out.ctypes.data) != 0:
            raise OracleError("bad rmax")
        return out

    def faults_strat(self, r, seed, shot):
        """Per-site fault outcome (or -1) of one shot conditioned on r faults."""
        out = np.zeros(max(self.nsites, 1), dtype=np.int32)
        rc = lib().oracle_faults_strat(self._h, r, seed, shot, out.ctypes.data)
        if rc:
            raise OracleError("stratum of %d faults: error %d" % (r, rc))
        return out[: self.nsites]

    def strat_survival(self, s, j, t):
        """P(next fault at or after site t | s faults left among sites j..N-1)."""
        return float(lib().oracle_strat_survival(self._h, s, j, t))

    def trace(self, seed=0, shot=0, forced_m=None, forced_faults=None):
        """Run one shot and return everything it produced (dict)."""
        ne, nr = max(self.nevents, 1), max(self.nrec, 1)
        probs = np.zeros(ne)
        ev_m = np.zeros(ne, np.uint8)
        recs = np.zeros(nr, np.uint8)
        dets = np.zeros(max(self.ndet, 1), np.uint8)
        obs = np.zeros(max(self.nobs, 1), np.uint8)
        phi = np.zeros(2 << self.kmax)
        slots = np.zeros(self.kmax + 1, np.int32)
        k = ctypes.c_int()
        gamma = np.zeros(2)
        faults = np.zeros(max(self.nsites, 1), np.int32)
        frame = np.zeros(4 * self.nq, np.uint8)
        expvals = np.zeros(max(self.nprobes, 1))
        fm = None if forced_m is None else np.ascontiguousarray(forced_m, dtype=np.uint8)
        ff = None if forced_faults is None else np.ascontiguousarray(forced_faults, dtype=np.int32)
        rc = lib().oracle_trace(self._h, seed, shot,
                                None if fm is None else fm.ctypes.data, None if ff is None else ff.ctypes.data,
                                probs.ctypes.data, ev_m.ctypes.data, recs.ctypes.data, dets.ctypes.data,
                                obs.ctypes.data, phi.ctypes.data, slots.ctypes.data, ctypes.addressof(k),
                                gamma.ctypes.data, faults.ctypes.data, frame.ctypes.data, expvals.ctypes.data)
        kk = k.value
        return dict(error=rc, probs=probs[: self.nevents], m=ev_m[: self.nevents], recs=recs[: self.nrec],
                    dets=dets[: self.ndet], obs=obs[: self.nobs],
                    phi=(phi[0::2] + 1j * phi[1::2])[: 1 << kk], slots=slots[:kk], k=kk,
                    gamma=complex(gamma[0], gamma[1]), faults=faults[: self.nsites],
                    frame=frame.reshape(4, self.nq), expvals=expvals[: self.nprobes])

    def sample(self, shots, seed=0, offset=0, threads=1, expvals=False, faults=None):
        """Bit-packed record-major outputs (meas, det, obs), each [count, ceil(shots/64)] uint64,
        and with expvals=True also the probes' values [nprobes, shots] (float64).
        faults=r: every shot conditioned on exactly r faults (stratified)."""
        words = (shots + 63) // 64
        meas = np.zeros((max(self.nrec, 1), max(words, 1)), np.uint64)
        det = np.zeros((max(self.ndet, 1), max(words, 1)), np.uint64)
        obs = np.zeros((max(self.nobs, 1), max(words, 1)), np.uint64)
        ev = np.zeros((max(self.nprobes, 1), max(shots, 1))) if expvals else None
        rc = lib().oracle_sample(self._h, shots, seed, offset, threads, meas.ctypes.data, det.ctypes.data,
                                 obs.ctypes.data, None if ev is None else ev.ctypes.data,
                                 -1 if faults is None else int(faults))
        if rc:
            raise OracleError("oracle sample error %d" % rc)
        out = (meas[: self.nrec, :words], det[: self.ndet, :words], obs[: self.nobs, :words])
        return out + (ev[: self.nprobes, :shots],) if expvals else out
