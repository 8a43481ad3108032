"""ctypes binding of libmpc3.so (include/mpc3.h): argument marshalling only.

Every step of the protocol runs in the library's HIP kernels; torch provides device
memory (int64 tensors used as raw 64-bit words) and the stream.  The library must be
built (``python -m paper_2411_09287_amd.build``); loading fails loudly otherwise.
"""
import ctypes
import functools
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpc3.so")

OK, E_ARG, E_SHAPE, E_NOMEM, E_ABORTED, E_UNVERIFIED, E_HIP, E_STATE, E_LIMIT = 0, -1, -2, -3, -4, -5, -6, -7, -8
VARIANT_U64, VARIANT_LIMB_I8, VARIANT_AUTO = 0, 1, 2
R_NETWORK = -2
PH_OFFLINE, PH_ONLINE, PH_VERIFY_OFFLINE, PH_VERIFY_ONLINE = 0, 1, 2, 3
VERIFY_INNER, VERIFY_TRUNC, VERIFY_MULT, VERIFY_NONLINEAR, VERIFY_ALL = 1, 2, 4, 8, 15
(SITE_INNER_GAMMA2, SITE_INNER_M1, SITE_TRUNC_GAMMA2, SITE_TRUNC_M1, SITE_MULT_GAMMA2, SITE_VER_H0_M1,
 SITE_VER_H2_GAMMA2, SITE_VER_DELTA_M1, SITE_REC_R1, SITE_AND_GAMMA2, SITE_EDA_W_M1) = range(1, 12)
MSG_GAMMA2, MSG_M1, MSG_M2 = 0, 1, 2
(LOG_R, LOG_Z, LOG_ZETA, LOG_H0_M1, LOG_H0_M2, LOG_H0_G2, LOG_H2_M1, LOG_H2_M2, LOG_H2_G2, LOG_DELTA,
 LOG_DELTA_M1, LOG_DELTA_M2, LOG_DELTA_G2) = range(13)


class Share(ctypes.Structure):
    _fields_ = [("m", ctypes.c_void_p), ("r1", ctypes.c_void_p), ("r2", ctypes.c_void_p),
                ("rows", ctypes.c_int64), ("cols", ctypes.c_int64)]


class TruncPair(ctypes.Structure):
    _fields_ = [("rx", Share), ("rz", Share), ("t", ctypes.c_int32), ("n", ctypes.c_int64),
                ("id", ctypes.c_uint64)]


class Comm(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_uint64 * 36), ("rounds", ctypes.c_uint32 * 4)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
SIGNATURES = {
    "mpc3_ctx_create": (_I, [_P, _I, _I, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "mpc3_ctx_destroy": (_I, [_P]),
    "mpc3_trim": (_I, [_P, ctypes.POINTER(_I64)]),
    "mpc3_set_variant": (_I, [_P, _I]),
    "mpc3_set_chunk": (_I, [_P, _I64]),
    "mpc3_autotune": (_I, [_P, _I64, _I64, _I64, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double)]),
    "mpc3_autotune_launch": (_I, [_P, _I64, _I64, _I64, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]),
    "mpc3_set_launch": (_I, [_P, _I64, _I64, _I64, _I, _I, _I]),
    "mpc3_set_verify_chunks": (_I, [_P, _I64, _I64]),
    "mpc3_set_network": (_I, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "mpc3_keep_messages": (_I, [_P, _I]),
    "mpc3_encode": (_I, [_P, _P, _I64, _P]),
    "mpc3_decode": (_I, [_P, _P, _I64, _P]),
    "mpc3_share": (_I, [_P, _I, _P, ctypes.POINTER(Share)]),
    "mpc3_trunc_pair": (_I, [_P, _I64, _I, ctypes.POINTER(TruncPair)]),
    "mpc3_inner": (_I, [_P, ctypes.POINTER(Share), ctypes.POINTER(Share), ctypes.POINTER(TruncPair),
                        ctypes.POINTER(Share)]),
    "mpc3_inner_static": (_I, [_P, ctypes.POINTER(Share), ctypes.POINTER(Share), ctypes.POINTER(TruncPair),
                               ctypes.POINTER(Share)]),
    "mpc3_im2col": (_I, [_P, ctypes.POINTER(Share), _I, _I, _I, _I, _I, _I, _I, ctypes.POINTER(Share)]),
    "mpc3_inner_conv": (_I, [_P, ctypes.POINTER(Share), _I, _I, _I, _I, _I, _I, _I, _I, ctypes.POINTER(Share),
                             ctypes.POINTER(Share), ctypes.POINTER(TruncPair), ctypes.POINTER(Share)]),
    "mpc3_im2col_strided": (_I, [_P, ctypes.POINTER(Share), _I, _I, _I, _I, _I, _I, _I, _I, ctypes.POINTER(Share)]),
    "mpc3_sumpool2": (_I, [_P, ctypes.POINTER(Share), _I, _I, _I, _I, ctypes.POINTER(Share)]),
    "mpc3_mult": (_I, [_P, ctypes.POINTER(Share), ctypes.POINTER(Share), ctypes.POINTER(Share)]),
    "mpc3_edabits": (_I, [_P, _I64, ctypes.POINTER(Share), ctypes.POINTER(Share)]),
    "mpc3_dabits": (_I, [_P, _I64, ctypes.POINTER(Share), ctypes.POINTER(Share)]),
    "mpc3_relu": (_I, [_P, ctypes.POINTER(Share), ctypes.POINTER(Share)]),
    "mpc3_maxpool2": (_I, [_P, ctypes.POINTER(Share), _I, _I, _I, _I, ctypes.POINTER(Share)]),
    "mpc3_trunc": (_I, [_P, ctypes.POINTER(TruncPair), ctypes.POINTER(Share), ctypes.POINTER(Share)]),
    "mpc3_capture_begin": (_I, [_P]),
    "mpc3_capture_end": (_I, [_P, ctypes.POINTER(_I)]),
    "mpc3_graph_launch": (_I, [_P, _I]),
    "mpc3_graph_nodes": (_I, [_P, _I, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "mpc3_graph_destroy": (_I, [_P, _I]),
    "mpc3_verify": (_I, [_P, _I, _I, ctypes.POINTER(_I)]),
    "mpc3_verify_begin": (_I, [_P, _I, _I]),
    "mpc3_verify_end": (_I, [_P, ctypes.POINTER(_I)]),
    "mpc3_reconstruct": (_I, [_P, ctypes.POINTER(Share), _I, _P]),
    "mpc3_comm_stats": (_I, [_P, ctypes.POINTER(Comm)]),
    "mpc3_inject": (_I, [_P, _I, _I64, _U64]),
    "mpc3_message": (_I, [_P, _I, _I, _P, _I64]),
    "mpc3_verify_log": (_I, [_P, _I64, _I, _I, _P, ctypes.POINTER(_I), ctypes.POINTER(_I64)]),
    "mpc3_profile": (_I, [_P, _I]),
    "mpc3_profile_read": (_I, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64),
                                ctypes.POINTER(ctypes.c_double)]),
    "mpc3_last_error": (_I, [_P, ctypes.POINTER(_I), ctypes.c_char_p, ctypes.c_size_t]),
    "mpc3_strerror": (ctypes.c_char_p, [_I]),
}

_lib = None


def lib():
    """Load libmpc3.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2411_09287_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class Mpc3Error(RuntimeError):
    def __init__(self, code, where, detail=""):
        self.code = code
        super().__init__(f"{where}: {lib().mpc3_strerror(code).decode()} ({code}){detail}")


def _ck(code, where, ctx=None):
    if code != OK:
        detail = ""
        if ctx is not None and code == E_HIP:
            hip = ctypes.c_int(0)
            buf = ctypes.create_string_buffer(512)
            lib().mpc3_last_error(ctx, ctypes.byref(hip), buf, 512)
            detail = f" [hipError {hip.value} at {buf.value.decode()}]"
        raise Mpc3Error(code, where, detail)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def to_words(a, device="cuda"):
    """uint64 numpy array -> int64 tensor on the device (same 64-bit patterns)."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
    return torch.from_numpy(a.view(np.int64)).to(device)


def from_words(t):
    """int64 tensor -> uint64 numpy array."""
    return t.detach().cpu().numpy().view(np.uint64)


def _planes(k, rows, cols, device):
    """k planes of rows x cols int64 words carved from one allocation, each starting on a
    256-byte boundary."""
    n = rows * cols
    stride = -(-n // 32) * 32
    base = torch.empty(max(k * stride, 1), dtype=torch.int64, device=device)
    return [base[p * stride:p * stride + n].view(rows, cols) for p in range(k)]


class DShare:
    """<v> on the device: three int64 tensors of one shape (m, [r]_1, [r]_2)."""

    def __init__(self, m, r1, r2):
        self.m, self.r1, self.r2 = m, r1, r2

    @classmethod
    def empty(cls, rows, cols, device="cuda"):
        return cls(*_planes(3, rows, cols, device))

    @property
    def rows(self):
        return self.m.shape[0]

    @property
    def cols(self):
        return self.m.shape[1] if self.m.dim() > 1 else 1

    def c(self):
        return Share(self.m.data_ptr(), self.r1.data_ptr(), self.r2.data_ptr(), self.rows, self.cols)

    def numpy(self):
        return tuple(from_words(t) for t in (self.m, self.r1, self.r2))


class DPair:
    """Truncation pair: planes of <r_x> and <r_z> (n words each) plus the C struct."""

    def __init__(self, n, device="cuda"):
        pl = _planes(6, n, 1, device)
        self.rx = DShare(*pl[:3])
        self.rz = DShare(*pl[3:])
        self.s = TruncPair(self.rx.c(), self.rz.c(), 0, n, 0)

    @property
    def n(self):
        return self.s.n

    @property
    def t(self):
        return self.s.t


def _on_stream(fn):
    """Run a Context method with the context's stream current, so that the tensors it
    allocates belong to the stream its launches are ordered on (torch's caching allocator
    reuses a freed block on the stream it was allocated on).  Input tensors must be ready
    on that stream."""
    @functools.wraps(fn)
    def run(self, *a, **k):
        if torch.cuda.current_stream(self.device) == self._stream:
            return fn(self, *a, **k)
        with torch.cuda.stream(self._stream):
            return fn(self, *a, **k)
    return run


class Context:
    """One three-party context on a torch stream (the current one by default)."""

    def __init__(self, master_seed, d=64, frac_bits=13, workspace_bytes=0, device="cuda", stream=None):
        self.device = device
        self.frac_bits = frac_bits
        seed = (ctypes.c_uint8 * 32).from_buffer_copy(bytes(master_seed))
        st = stream if stream is not None else torch.cuda.current_stream(device)
        self._stream = st
        h = ctypes.c_void_p()
        _ck(lib().mpc3_ctx_create(seed, d, frac_bits, workspace_bytes, ctypes.c_void_p(st.cuda_stream),
                                  ctypes.byref(h)), "mpc3_ctx_create")
        self.h = h
        # operands the context still points at, per kind of pending product
        self._keep = {VERIFY_INNER: [], VERIFY_TRUNC: [], VERIFY_MULT: [], VERIFY_NONLINEAR: []}

    def close(self):
        if self.h:
            lib().mpc3_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- configuration -------------------------------------------------------
    def set_variant(self, v):
        _ck(lib().mpc3_set_variant(self.h, v), "mpc3_set_variant", self.h)

    def autotune(self, M, K, N, reps=3):
        ch, a, b = ctypes.c_int(0), ctypes.c_double(0), ctypes.c_double(0)
        _ck(lib().mpc3_autotune(self.h, M, K, N, reps, ctypes.byref(ch), ctypes.byref(a), ctypes.byref(b)),
            "mpc3_autotune", self.h)
        return ch.value, a.value, b.value

    def autotune_launch(self, M, K, N, reps=5):
        """Launch-shape autotuner of the limb kernel: ((ns, rb, split), ms_default, ms_best)."""
        sh = (ctypes.c_int * 3)()
        a, b = ctypes.c_double(0), ctypes.c_double(0)
        _ck(lib().mpc3_autotune_launch(self.h, M, K, N, reps, sh, ctypes.byref(a), ctypes.byref(b)),
            "mpc3_autotune_launch", self.h)
        return (sh[0], sh[1], sh[2]), a.value, b.value

    def set_launch(self, M, K, N, ns=0, rb=0, split=0):
        _ck(lib().mpc3_set_launch(self.h, M, K, N, ns, rb, split), "mpc3_set_launch", self.h)

    def set_chunk(self, t):
        _ck(lib().mpc3_set_chunk(self.h, t), "mpc3_set_chunk", self.h)

    def set_verify_chunks(self, mult_triples=0, edabit_rows=0):
        _ck(lib().mpc3_set_verify_chunks(self.h, mult_triples, edabit_rows), "mpc3_set_verify_chunks", self.h)

    def set_network(self, rtt_ms, mbit_per_s, gpu_round_ms=0.1):
        _ck(lib().mpc3_set_network(self.h, rtt_ms, mbit_per_s, gpu_round_ms), "mpc3_set_network", self.h)

    def keep_messages(self, on=True):
        _ck(lib().mpc3_keep_messages(self.h, int(on)), "mpc3_keep_messages", self.h)

    # -- protocol --------------------------------------------------------------
    @property
    def stream(self):
        """The torch stream the context's launches are ordered on."""
        return self._stream

    @_on_stream
    def encode(self, x, out=None):
        x = x.to(self.device, torch.float64).contiguous()
        if out is None:
            out = torch.empty(x.shape, dtype=torch.int64, device=self.device)
        _ck(lib().mpc3_encode(self.h, _ptr(x), x.numel(), _ptr(out)), "mpc3_encode", self.h)
        return out

    @_on_stream
    def decode(self, v):
        out = torch.empty(v.shape, dtype=torch.float64, device=self.device)
        _ck(lib().mpc3_decode(self.h, _ptr(v), v.numel(), _ptr(out)), "mpc3_decode", self.h)
        return out

    @_on_stream
    def share(self, x, owner=0, out=None):
        x = x.contiguous()
        rows = x.shape[0] if x.dim() else 1
        cols = x.numel() // rows if rows else 0
        if out is None:
            out = DShare.empty(rows, cols, self.device)
        s = out.c()
        _ck(lib().mpc3_share(self.h, owner, _ptr(x), ctypes.byref(s)), "mpc3_share", self.h)
        return out

    @_on_stream
    def trunc_pair(self, n, t, out=None):
        p = out if out is not None else DPair(n, self.device)
        _ck(lib().mpc3_trunc_pair(self.h, n, t, ctypes.byref(p.s)), "mpc3_trunc_pair", self.h)
        self._keep[VERIFY_TRUNC].append(p)
        return p

    @_on_stream
    def inner(self, X, W, pair=None, out=None):
        Z = out if out is not None else DShare.empty(X.rows, W.cols, self.device)
        xs, ws, zs = X.c(), W.c(), Z.c()
        _ck(lib().mpc3_inner(self.h, ctypes.byref(xs), ctypes.byref(ws),
                             ctypes.byref(pair.s) if pair is not None else None, ctypes.byref(zs)), "mpc3_inner", self.h)
        self._keep[VERIFY_INNER].append((X, W, Z))
        return Z

    @_on_stream
    def inner_static(self, X, W, pair=None, out=None):
        """mpc3_inner_static: Pi_Inner with the library's fixed device workspace (no allocation
        inside the call; Z must be given or is allocated here, before the call)."""
        Z = out if out is not None else DShare.empty(X.rows, W.cols, self.device)
        xs, ws, zs = X.c(), W.c(), Z.c()
        _ck(lib().mpc3_inner_static(self.h, ctypes.byref(xs), ctypes.byref(ws),
                                    ctypes.byref(pair.s) if pair is not None else None, ctypes.byref(zs)),
            "mpc3_inner_static", self.h)
        self._keep[VERIFY_INNER].append((X, W, Z))
        return Z

    @_on_stream
    def inner_conv(self, x, B, H, W, C, KH, KW, pad, Wt, pair=None, ld=None, stride=1, cols=None, out=None):
        """mpc3_inner_conv: Pi_Inner of the lowering of x (Wt.rows = ld >= KH KW C columns) with
        Wt, the product verified from x.  cols=None lets the library lower implicitly in the
        product kernel or into memory of its own; a DShare cols receives the lowering.
        Returns Z."""
        OH, OW = (H + 2 * pad - KH) // stride + 1, (W + 2 * pad - KW) // stride + 1
        if ld is not None and ld != Wt.rows:
            raise ValueError("ld must equal Wt.rows")
        Z = out if out is not None else DShare.empty(B * OH * OW, Wt.cols, self.device)
        xs, ws, zs = x.c(), Wt.c(), Z.c()
        cs = cols.c() if cols is not None else None
        _ck(lib().mpc3_inner_conv(self.h, ctypes.byref(xs), B, H, W, C, KH, KW, pad, stride,
                                  ctypes.byref(cs) if cs is not None else None,
                                  ctypes.byref(ws), ctypes.byref(pair.s) if pair is not None else None,
                                  ctypes.byref(zs)), "mpc3_inner_conv", self.h)
        self._keep[VERIFY_INNER].append((x, cols, Wt, Z))
        return Z

    @_on_stream
    def im2col(self, x, B, H, W, C, KH, KW, pad, ld=None, stride=1, out=None):
        """ld (>= KH KW C): row width of the result, the extra columns zero."""
        OH, OW = (H + 2 * pad - KH) // stride + 1, (W + 2 * pad - KW) // stride + 1
        cols = out if out is not None else DShare.empty(B * OH * OW, ld or KH * KW * C, self.device)
        xs, cs = x.c(), cols.c()
        if stride == 1:
            _ck(lib().mpc3_im2col(self.h, ctypes.byref(xs), B, H, W, C, KH, KW, pad, ctypes.byref(cs)), "mpc3_im2col",
                self.h)
        else:
            _ck(lib().mpc3_im2col_strided(self.h, ctypes.byref(xs), B, H, W, C, KH, KW, pad, stride, ctypes.byref(cs)),
                "mpc3_im2col_strided", self.h)
        return cols

    @_on_stream
    def sumpool2(self, x, B, H, W, C, out=None):
        if out is None:
            out = DShare.empty(B, (H // 2) * (W // 2) * C, self.device)
        xs, os_ = x.c(), out.c()
        _ck(lib().mpc3_sumpool2(self.h, ctypes.byref(xs), B, H, W, C, ctypes.byref(os_)), "mpc3_sumpool2", self.h)
        return out

    @_on_stream
    def mult(self, a, b):
        c = DShare.empty(a.rows, a.cols, self.device)
        sa, sb, sc = a.c(), b.c(), c.c()
        _ck(lib().mpc3_mult(self.h, ctypes.byref(sa), ctypes.byref(sb), ctypes.byref(sc)), "mpc3_mult", self.h)
        self._keep[VERIFY_MULT].append((a, b, c))
        return c

    @_on_stream
    def edabits(self, n):
        """(arith, bits): <r>^l and <r[0..63]>^1 of n random edaBits (n words per plane each)."""
        a, b = DShare.empty(n, 1, self.device), DShare.empty(n, 1, self.device)
        sa, sb = a.c(), b.c()
        _ck(lib().mpc3_edabits(self.h, n, ctypes.byref(sa), ctypes.byref(sb)), "mpc3_edabits", self.h)
        return a, b

    @_on_stream
    def dabits(self, n):
        a, b = DShare.empty(n, 1, self.device), DShare.empty(n, 1, self.device)
        sa, sb = a.c(), b.c()
        _ck(lib().mpc3_dabits(self.h, n, ctypes.byref(sa), ctypes.byref(sb)), "mpc3_dabits", self.h)
        return a, b

    @_on_stream
    def relu(self, x):
        out = DShare.empty(x.rows, x.cols, self.device)
        xs, os_ = x.c(), out.c()
        _ck(lib().mpc3_relu(self.h, ctypes.byref(xs), ctypes.byref(os_)), "mpc3_relu", self.h)
        self._keep[VERIFY_MULT].append((x, out))
        return out

    @_on_stream
    def maxpool2(self, x, B, H, W, C):
        out = DShare.empty(B, (H // 2) * (W // 2) * C, self.device)
        xs, os_ = x.c(), out.c()
        _ck(lib().mpc3_maxpool2(self.h, ctypes.byref(xs), B, H, W, C, ctypes.byref(os_)), "mpc3_maxpool2", self.h)
        self._keep[VERIFY_MULT].append((x, out))
        return out

    @_on_stream
    def trunc(self, pair, Z, out=None):
        if out is None:
            out = DShare.empty(Z.rows, Z.cols, self.device)
        zs, os_ = Z.c(), out.c()
        _ck(lib().mpc3_trunc(self.h, ctypes.byref(pair.s), ctypes.byref(zs), ctypes.byref(os_)), "mpc3_trunc", self.h)
        return out

    # -- recorded forward passes (HIP graphs) -------------------------------------
    def capture_begin(self):
        _ck(lib().mpc3_capture_begin(self.h), "mpc3_capture_begin", self.h)

    def capture_end(self):
        gid = ctypes.c_int(0)
        _ck(lib().mpc3_capture_end(self.h, ctypes.byref(gid)), "mpc3_capture_end", self.h)
        return gid.value

    def graph_launch(self, gid):
        _ck(lib().mpc3_graph_launch(self.h, gid), "mpc3_graph_launch", self.h)

    def graph_nodes(self, gid):
        k, o = ctypes.c_int64(0), ctypes.c_int64(0)
        _ck(lib().mpc3_graph_nodes(self.h, gid, ctypes.byref(k), ctypes.byref(o)), "mpc3_graph_nodes", self.h)
        return k.value, o.value

    def graph_destroy(self, gid):
        _ck(lib().mpc3_graph_destroy(self.h, gid), "mpc3_graph_destroy", self.h)

    def verify(self, R=-1, kinds=VERIFY_ALL):
        ok = ctypes.c_int(0)
        _ck(lib().mpc3_verify(self.h, R, kinds, ctypes.byref(ok)), "mpc3_verify", self.h)
        for k in self._keep:
            if kinds & k:
                self._keep[k] = []
        return bool(ok.value)

    def verify_begin(self, R=-1, kinds=VERIFY_ALL):
        """mpc3_verify_begin: enqueue the verification and return; verify_end() gives ok."""
        _ck(lib().mpc3_verify_begin(self.h, R, kinds), "mpc3_verify_begin", self.h)
        self._inflight = [self._keep[k] for k in self._keep if kinds & k]
        for k in self._keep:
            if kinds & k:
                self._keep[k] = []

    def verify_end(self):
        ok = ctypes.c_int(0)
        _ck(lib().mpc3_verify_end(self.h, ctypes.byref(ok)), "mpc3_verify_end", self.h)
        self._inflight = []
        return bool(ok.value)

    @_on_stream
    def reconstruct(self, X, to_party=-1, out=None):
        if out is None:
            out = torch.empty(X.m.shape, dtype=torch.int64, device=self.device)
        xs = X.c()
        _ck(lib().mpc3_reconstruct(self.h, ctypes.byref(xs), to_party, _ptr(out)), "mpc3_reconstruct", self.h)
        return out

    def last_error(self):
        """(code, hipError_t, where) of the last failed call on this context."""
        hip = ctypes.c_int(0)
        buf = ctypes.create_string_buffer(512)
        code = lib().mpc3_last_error(self.h, ctypes.byref(hip), buf, 512)
        return code, hip.value, buf.value.decode()

    def comm_stats(self):
        c = Comm()
        _ck(lib().mpc3_comm_stats(self.h, ctypes.byref(c)), "mpc3_comm_stats", self.h)
        b = np.array(list(c.bytes), dtype=np.uint64).reshape(4, 3, 3)
        return b, list(c.rounds)

    def inject(self, site, index, e):
        _ck(lib().mpc3_inject(self.h, site, index, e & ((1 << 64) - 1)), "mpc3_inject", self.h)

    @_on_stream
    def message(self, kind, which, n):
        out = torch.empty(n, dtype=torch.int64, device=self.device)
        _ck(lib().mpc3_message(self.h, kind, which, _ptr(out), n), "mpc3_message", self.h)
        return out

    def trim(self):
        """Return the device memory the context caches between calls (workspaces, pooled
        lowering buffers); the bytes returned."""
        n = ctypes.c_int64(0)
        _ck(lib().mpc3_trim(self.h, ctypes.byref(n)), "mpc3_trim", self.h)
        return n.value

    def profile(self, on=True):
        _ck(lib().mpc3_profile(self.h, int(on)), "mpc3_profile", self.h)

    def profile_read(self):
        t, n, w = ctypes.c_double(0), ctypes.c_int64(0), ctypes.c_double(0)
        _ck(lib().mpc3_profile_read(self.h, ctypes.byref(t), ctypes.byref(n), ctypes.byref(w)), "mpc3_profile_read", self.h)
        return t.value, n.value, w.value

    def verify_log(self, instance, slot, rnd=0):
        buf = (ctypes.c_uint64 * 64)()
        R = ctypes.c_int(0)
        dim = ctypes.c_int64(0)
        _ck(lib().mpc3_verify_log(self.h, instance, slot, rnd, buf, ctypes.byref(R), ctypes.byref(dim)),
            "mpc3_verify_log", self.h)
        return np.array(list(buf), dtype=np.uint64), R.value, dim.value
