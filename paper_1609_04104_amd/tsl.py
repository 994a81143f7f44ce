"""Python binding of libtsl (include/tsl.h): argument marshalling only.

Every step of the method runs in the HIP library; this module checks tensor
dtypes, shapes and devices, passes raw device pointers and the current HIP
stream, and turns negative return codes into ``TslError``.  It never computes
anything itself and raises if the library is not built.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsl.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTPD, ENONFINITE, EBUSY, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
STEP_MM, STEP_CONST = 0, 1
MAX_R = 128
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ENOTPD: "ENOTPD",
          ENONFINITE: "ENONFINITE", EBUSY: "EBUSY", EUNSUPPORTED: "EUNSUPPORTED"}

EXPORTS = [
    "tsl_opts_default", "tsl_size_supported", "tsl_footprint", "tsl_open", "tsl_close",
    "tsl_push_lines", "tsl_push_points", "tsl_push_frame", "tsl_sample_lines", "tsl_step_many",
    "tsl_step_many_noalloc", "tsl_epochs", "tsl_sample_points", "tsl_open_coils", "tsl_push_coils",
    "tsl_output_tile", "tsl_set_output_tile",
    "tsl_step_many_timed", "tsl_batch_create", "tsl_batch_launch", "tsl_batch_destroy", "tsl_status",
    "tsl_get_factors", "tsl_get_state", "tsl_set_state", "tsl_shape", "tsl_fft2",
    "tsl_pool_create", "tsl_pool_destroy", "tsl_pool_used", "tsl_open_in_pool",
    "tsl_last_error", "tsl_selftest_codelets",
]


class TslError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("step_mode", ctypes.c_int), ("mu", ctypes.c_double), ("allow_lambda0", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint64), ("line_route", ctypes.c_int),
                ("synth_bf16", ctypes.c_int)]


N_PHASES = 7
PHASES = ["partial Grams", "ridge solve + step size", "synthesis + row pass", "column pass + residual",
          "row inverse + A grad", "factor updates + F_l A, F_r B",
          "output synthesis + row draw"]
ROUTE_KSPACE, ROUTE_FRAME = 0, 1
BATCH_GRAPH = 1


class Frame(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int), ("rows", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("X_out", ctypes.c_void_p), ("A_out", ctypes.c_void_p),
                ("B_out", ctypes.c_void_p), ("gamma_out", ctypes.c_void_p), ("n_rows_dev", ctypes.c_void_p),
                ("y_full", ctypes.c_int), ("K_next", ctypes.c_int), ("rows_next", ctypes.c_void_p),
                ("n_next", ctypes.c_void_p), ("info_out", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded libtsl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1609_04104_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        P = ctypes.POINTER
        sig = {
            "tsl_opts_default": (None, [P(Opts)]),
            "tsl_size_supported": (i, [i]),
            "tsl_footprint": (i, [i, i, i, P(sz)]),
            "tsl_open": (i, [P(vp), i, i, i, d, P(Opts), vp, vp, vp]),
            "tsl_close": (i, [vp]),
            "tsl_push_lines": (i, [vp, i, vp, vp, vp, vp, vp, vp, vp]),
            "tsl_push_points": (i, [vp, vp, vp, vp, vp, vp, vp, vp]),
            "tsl_sample_lines": (i, [vp, i, vp, vp, vp, vp, vp]),
            "tsl_push_frame": (i, [vp, P(Frame), vp]),
            "tsl_epochs": (i, [vp, i, P(Frame), i, vp, vp]),
            "tsl_sample_points": (i, [vp, i, vp, vp, vp, vp]),
            "tsl_open_coils": (i, [P(vp), i, i, i, i, d, P(Opts), vp, vp, vp, vp]),
            "tsl_output_tile": (i, [i, i, i, i]),
            "tsl_set_output_tile": (i, [i, i, i, i, i]),
            "tsl_push_coils": (i, [vp, i, vp, vp, vp, vp, vp, vp, vp]),
            "tsl_step_many": (i, [P(vp), i, P(Frame), vp]),
            "tsl_step_many_noalloc": (i, [P(vp), i, P(Frame), vp]),
            "tsl_step_many_timed": (i, [P(vp), i, P(Frame), P(d), vp]),
            "tsl_batch_create": (i, [P(vp), i, P(Frame), i, P(vp)]),
            "tsl_batch_launch": (i, [vp, vp]),
            "tsl_batch_destroy": (i, [vp]),
            "tsl_status": (i, [vp, i]),
            "tsl_get_factors": (i, [vp, vp, vp, vp, vp, vp]),
            "tsl_get_state": (i, [vp, vp, P(sz)]),
            "tsl_set_state": (i, [vp, vp, sz]),
            "tsl_shape": (i, [vp, P(i), P(i), P(i)]),
            "tsl_fft2": (i, [i, i, i, vp, vp, i, vp]),
            "tsl_pool_create": (i, [P(vp), sz]),
            "tsl_pool_destroy": (i, [vp]),
            "tsl_pool_used": (i, [vp, P(sz), P(sz)]),
            "tsl_open_in_pool": (i, [vp, P(vp), i, i, i, d, P(Opts), vp, vp, vp]),
            "tsl_last_error": (ctypes.c_char_p, []),
            "tsl_selftest_codelets": (d, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise TslError(rc, lib().tsl_last_error().decode())
    return rc


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtype, shape=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor of the given dtype/shape."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def size_supported(n):
    return bool(lib().tsl_size_supported(int(n)))


def footprint(n1, n2, r):
    b = ctypes.c_size_t(0)
    _check(lib().tsl_footprint(n1, n2, r, ctypes.byref(b)))
    return b.value


OUT_TILES = {0: "128x64", 1: "64x64", 2: "128x128"}


def output_tile(n1, n2, r, count):
    """The output-synthesis block tile a launch of `count` frames uses now."""
    return OUT_TILES[_check(lib().tsl_output_tile(int(n1), int(n2), int(r), int(count)))]


def set_output_tile(n1, n2, r, count, tile):
    """Fixes the output-synthesis tile ("128x64", "64x64" or "128x128") of such launches."""
    code = {v: k for k, v in OUT_TILES.items()}[tile]
    _check(lib().tsl_set_output_tile(int(n1), int(n2), int(r), int(count), code))


def selftest_codelets():
    return float(lib().tsl_selftest_codelets())


SYNTH = {"fp32": 0, "bf16": 1, "bf16x3": 2}


def make_opts(step_mode="mm", mu=0.0, allow_lambda0=False, seed=0, stream_id=0, route="kspace", synth="fp32"):
    o = Opts()
    lib().tsl_opts_default(ctypes.byref(o))
    o.synth_bf16 = SYNTH[synth]
    o.line_route = {"kspace": ROUTE_KSPACE, "frame": ROUTE_FRAME}[route]
    o.step_mode = {"mm": STEP_MM, "const": STEP_CONST}[step_mode]
    o.mu = float(mu)
    o.allow_lambda0 = int(bool(allow_lambda0))
    o.seed = int(seed) & (2**64 - 1)
    o.stream_id = int(stream_id) & (2**64 - 1)
    return o


class Pool:
    """Device-byte budget for admitting sequences (tsl_pool_*)."""

    def __init__(self, budget_bytes):
        h = ctypes.c_void_p()
        _check(lib().tsl_pool_create(ctypes.byref(h), int(budget_bytes)))
        self.h = h

    def used(self):
        u, b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().tsl_pool_used(self.h, ctypes.byref(u), ctypes.byref(b)))
        return u.value, b.value

    def destroy(self):
        if self.h:
            _check(lib().tsl_pool_destroy(self.h))
            self.h = None


class Sequence:
    """One scan's resident state (tsl_open ... tsl_close)."""

    def __init__(self, n1, n2, r, lam, A0, B0, step_mode="mm", mu=0.0, allow_lambda0=False,
                 seed=0, stream_id=0, pool=None, stream=None, route="kspace", synth="fp32"):
        self.n1, self.n2, self.r = int(n1), int(n2), int(r)
        self.opts = make_opts(step_mode, mu, allow_lambda0, seed, stream_id, route, synth)
        a = _dev(A0, torch.complex64, (n1, r), "A0")
        b = _dev(B0, torch.complex64, (n2, r), "B0")
        h = ctypes.c_void_p()
        if pool is None:
            _check(lib().tsl_open(ctypes.byref(h), n1, n2, r, float(lam), ctypes.byref(self.opts), a, b,
                                  _stream(stream)))
        else:
            _check(lib().tsl_open_in_pool(pool.h, ctypes.byref(h), n1, n2, r, float(lam),
                                          ctypes.byref(self.opts), a, b, _stream(stream)))
        self.h = h

    # ---------------------------------------------------------------- per frame
    def _outs(self, X_out, A_out, B_out, gamma_out):
        return (_dev(X_out, torch.complex64, (self.n1, self.n2), "X_out"),
                _dev(A_out, torch.complex64, (self.n1, self.r), "A_out"),
                _dev(B_out, torch.complex64, (self.n2, self.r), "B_out"),
                _dev(gamma_out, torch.complex64, (self.r,), "gamma_out"))

    def push_lines(self, rows, y, X_out=None, A_out=None, B_out=None, gamma_out=None, stream=None):
        n = int(rows.shape[0])
        rp = _dev(rows, torch.int32, (n,), "rows")
        yp = _dev(y, torch.complex64, (n, self.n2), "y")
        _check(lib().tsl_push_lines(self.h, n, rp, yp, *self._outs(X_out, A_out, B_out, gamma_out),
                                    _stream(stream)))

    def push_points(self, mask, y, X_out=None, A_out=None, B_out=None, gamma_out=None, stream=None):
        mp = _dev(mask, torch.uint8, (self.n1, self.n2), "mask")
        yp = _dev(y, torch.complex64, (self.n1, self.n2), "y")
        _check(lib().tsl_push_points(self.h, mp, yp, *self._outs(X_out, A_out, B_out, gamma_out),
                                     _stream(stream)))

    def sample_lines(self, K, rows_out, n_out, draws_out=None, prefix_out=None, stream=None):
        _check(lib().tsl_sample_lines(self.h, int(K), _dev(rows_out, torch.int32, (K,), "rows_out"),
                                      _dev(n_out, torch.int32, (1,), "n_out"),
                                      _dev(draws_out, torch.int32, (K,), "draws_out"),
                                      _dev(prefix_out, torch.float64, (self.n1,), "prefix_out"),
                                      _stream(stream)))

    def sample_points(self, K, mask_out, n_out, draws_out=None, stream=None):
        """tsl_sample_points: the entries of frame t+1 drawn by eq. (13)."""
        _check(lib().tsl_sample_points(self.h, int(K), _dev(mask_out, torch.uint8, (self.n1, self.n2), "mask_out"),
                                       _dev(n_out, torch.int32, (1,), "n_out"),
                                       _dev(draws_out, torch.int32, (K,), "draws_out"), _stream(stream)))

    def frame(self, rows=None, y=None, mask=None, X_out=None, A_out=None, B_out=None, gamma_out=None,
              n_rows_dev=None, y_full=False, K_next=0, rows_next=None, n_next=None, info_out=None):
        """A tsl_frame for push_frame / step_many (keeps the tensors alive on the struct).

        rows: int32 [n] (or a capacity-sized buffer when n_rows_dev holds the count);
        y: [n, n2] samples, or [n1, n2] with y_full=True / a point mask;
        info_out: float64 [4] receiving alpha_t, alpha_bar_t, mu_t and the pivot
        ratio of the ridge Gram."""
        f = Frame()
        if mask is not None:
            f.mask = _dev(mask, torch.uint8, (self.n1, self.n2), "mask")
            f.y = _dev(y, torch.complex64, (self.n1, self.n2), "y")
        else:
            n = int(rows.shape[0])
            f.n_rows = n
            f.rows = _dev(rows, torch.int32, (n,), "rows")
            f.y_full = int(bool(y_full))
            f.y = _dev(y, torch.complex64, (self.n1, self.n2) if y_full else (n, self.n2), "y")
            f.n_rows_dev = _dev(n_rows_dev, torch.int32, (1,), "n_rows_dev")
        f.X_out, f.A_out, f.B_out, f.gamma_out = self._outs(X_out, A_out, B_out, gamma_out)
        if K_next:
            f.K_next = int(K_next)
            f.rows_next = _dev(rows_next, torch.int32, (int(K_next),), "rows_next")
            f.n_next = _dev(n_next, torch.int32, (1,), "n_next")
        f.info_out = _dev(info_out, torch.float64, (4,), "info_out")
        f._keep = (rows, y, mask, X_out, A_out, B_out, gamma_out, n_rows_dev, rows_next, n_next, info_out)
        return f

    def push(self, frame, stream=None):
        """tsl_push_frame with a Frame from self.frame(...)."""
        _check(lib().tsl_push_frame(self.h, ctypes.byref(frame), _stream(stream)))

    def epochs(self, frames, order, stream=None):
        """tsl_epochs: passes over the stored frames (Frames from self.frame(...));
        order is an integer array [E, T], each row a permutation of range(T)."""
        import numpy as np
        order = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
        if order.ndim != 2 or order.shape[1] != len(frames):
            raise ValueError("order must be [E, T] with T = len(frames)")
        fs = (Frame * len(frames))(*frames)
        _check(lib().tsl_epochs(self.h, len(frames), fs, order.shape[0], order.ctypes.data_as(ctypes.c_void_p),
                                _stream(stream)))

    # ---------------------------------------------------------------- state
    def status(self, clear=False):
        return lib().tsl_status(self.h, int(bool(clear)))

    def factors(self, A=None, B=None, Ahat=None, Bhat=None, stream=None):
        _check(lib().tsl_get_factors(self.h, _dev(A, torch.complex64, (self.n1, self.r), "A"),
                                     _dev(B, torch.complex64, (self.n2, self.r), "B"),
                                     _dev(Ahat, torch.complex64, (self.n1, self.r), "Ahat"),
                                     _dev(Bhat, torch.complex64, (self.n2, self.r), "Bhat"),
                                     _stream(stream)))

    def get_state(self):
        n = ctypes.c_size_t(0)
        _check(lib().tsl_get_state(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().tsl_get_state(self.h, buf, ctypes.byref(n)))
        return buf.raw[:n.value]

    def set_state(self, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().tsl_set_state(self.h, buf, len(blob)))

    def close(self):
        if getattr(self, "h", None):
            _check(lib().tsl_close(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_many(seqs, frames, stream=None):
    """One batched step: frames[i] (from Sequence.frame) for seqs[i]."""
    n = len(seqs)
    hs = (ctypes.c_void_p * n)(*[s.h for s in seqs])
    fs = (Frame * n)(*frames)
    _check(lib().tsl_step_many(hs, n, fs, _stream(stream)))


STATIC_MAX_FRAMES = 256


def step_many_noalloc(seqs, frames, stream=None):
    """tsl_step_many_noalloc: the batched step with its descriptors in the
    library's fixed device array (no device allocation; at most
    STATIC_MAX_FRAMES frames; calls that overlap on one GPU race)."""
    n = len(seqs)
    hs = (ctypes.c_void_p * n)(*[s.h for s in seqs])
    fs = (Frame * n)(*frames)
    _check(lib().tsl_step_many_noalloc(hs, n, fs, _stream(stream)))


class PreparedStep:
    """A batched step fixed once (tsl_batch_create): validated and its
    descriptors uploaded at construction, so that a launch only launches
    kernels -- directly (default), or by replaying a HIP graph captured at
    construction (graph=True).  The sequences and the frames' tensors must stay
    alive; closing one of the sequences makes launch() raise."""

    def __init__(self, seqs, frames, graph=False):
        n = len(seqs)
        hs = (ctypes.c_void_p * n)(*[s.h for s in seqs])
        fs = (Frame * n)(*frames)
        h = ctypes.c_void_p()
        _check(lib().tsl_batch_create(hs, n, fs, BATCH_GRAPH if graph else 0, ctypes.byref(h)))
        self.h = h
        self.n = n
        self._keep = (list(seqs), list(frames))

    def launch(self, stream=None):
        if self.h is None:
            raise TslError(EINVAL, "prepared step has been closed")
        _check(lib().tsl_batch_launch(self.h, _stream(stream)))

    def close(self):
        """Waits for the last launch and frees the descriptors and the graph."""
        h, self.h = self.h, None
        if h is not None:
            _check(lib().tsl_batch_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_many_timed(seqs, frames, phase_ms=None, stream=None):
    """Profiling form of step_many (no graph; waits).  Adds per-phase milliseconds
    to phase_ms (a list of N_PHASES floats) and returns it."""
    n = len(seqs)
    hs = (ctypes.c_void_p * n)(*[s.h for s in seqs])
    fs = (Frame * n)(*frames)
    acc = (ctypes.c_double * N_PHASES)(*(phase_ms or [0.0] * N_PHASES))
    _check(lib().tsl_step_many_timed(hs, n, fs, acc, _stream(stream)))
    return list(acc)


def fft2(x, out=None, inverse=False, stream=None):
    """Unitary 2-D transform of x [batch, n1, n2] or [n1, n2] (complex64, on the GPU)."""
    if out is None:
        out = torch.empty_like(x)
    shape = tuple(x.shape)
    if len(shape) == 2:
        batch, n1, n2 = 1, shape[0], shape[1]
    elif len(shape) == 3:
        batch, n1, n2 = shape
    else:
        raise ValueError("x must be [n1, n2] or [batch, n1, n2]")
    _check(lib().tsl_fft2(n1, n2, batch, _dev(x, torch.complex64, shape, "x"),
                          _dev(out, torch.complex64, shape, "out"), int(bool(inverse)), _stream(stream)))
    return out


class CoilSequence(Sequence):
    """A scan imaged by C coils with sensitivity maps H [C, n1, n2] (tsl_open_coils)."""

    def __init__(self, n1, n2, r, lam, A0, B0, H, step_mode="mm", mu=0.0, allow_lambda0=False, seed=0,
                 stream_id=0, stream=None, synth="fp32"):
        self.n1, self.n2, self.r = int(n1), int(n2), int(r)
        self.C = int(H.shape[0])
        self.opts = make_opts(step_mode, mu, allow_lambda0, seed, stream_id, "frame", synth)
        a = _dev(A0, torch.complex64, (n1, r), "A0")
        b = _dev(B0, torch.complex64, (n2, r), "B0")
        hp = _dev(H, torch.complex64, (self.C, n1, n2), "H")
        h = ctypes.c_void_p()
        _check(lib().tsl_open_coils(ctypes.byref(h), n1, n2, r, self.C, float(lam), ctypes.byref(self.opts), a, b,
                                    hp, _stream(stream)))
        self.h = h

    def push_coils(self, rows, y, X_out=None, A_out=None, B_out=None, gamma_out=None, stream=None):
        """rows: int32 [n]; y: complex64 [C, n, n2]."""
        n = int(rows.shape[0])
        rp = _dev(rows, torch.int32, (n,), "rows")
        yp = _dev(y, torch.complex64, (self.C, n, self.n2), "y")
        _check(lib().tsl_push_coils(self.h, n, rp, yp, *self._outs(X_out, A_out, B_out, gamma_out), _stream(stream)))
