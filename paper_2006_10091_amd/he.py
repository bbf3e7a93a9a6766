"""Python binding of libhe (include/he.h): argument marshalling only.

Device memory for ciphertexts, plaintexts and keys is allocated with torch and
handed to the library as raw pointers; every computation runs in the HIP
library.  There is no CPU fallback: importing this module fails loudly when
libhe.so has not been built.
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p

import numpy as np
# torch's HIP runtime must be the process's only one: load it before libhe.so,
# whose libamdhip64.so.7 dependency then resolves to the already-loaded copy.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhe.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libhe.so is not built (run __graft_entry__.build() or "
                      "python -m paper_2006_10091_amd.build); there is no fallback")

_lib = ctypes.CDLL(LIB_PATH)

STATUS = {0: "HE_OK", 1: "HE_EINVAL", 2: "HE_ENOMEM", 3: "HE_ELEVEL", 4: "HE_ESCALE", 5: "HE_EKEY",
          6: "HE_EDEVICE"}
HE_ENOMEM = 2  # a device allocation failed


class HEError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.he_strerror(status).decode()
        super().__init__("%s: %s (%s)" % (where, STATUS.get(status, status), msg))


class he_params(ctypes.Structure):
    _fields_ = [("log_n", c_int32), ("n_q", c_int32), ("n_special", c_int32), ("alpha", c_int32),
                ("log_delta", c_int32)]


class he_ct(ctypes.Structure):
    _fields_ = [("data", c_void_p), ("level", c_int32), ("reserved", c_int32), ("scale", c_double)]


he_pt = he_ct
he_ct3 = he_ct


class he_lr_request(ctypes.Structure):
    _fields_ = [("Z", POINTER(he_ct)), ("n_blocks", c_int32), ("W", POINTER(he_ct)), ("mask", POINTER(he_ct)),
                ("coef", POINTER(c_double)), ("eta_over_n", c_double), ("w_decay", c_double),
                ("W_out", POINTER(he_ct)), ("G_out", POINTER(he_ct))]


class he_op(ctypes.Structure):
    _fields_ = [("op", c_int32), ("steps", c_int32), ("x", he_ct), ("y", he_ct), ("out", he_ct)]


OP_MUL, OP_MUL_ROTATE, OP_ROTATE, OP_RESCALE, OP_ADD = 1, 2, 3, 4, 5


class he_ct_seeded(ctypes.Structure):
    _fields_ = [("b", c_void_p), ("level", c_int32), ("reserved", c_int32), ("scale", c_double), ("seed", c_uint64),
                ("index", c_uint32), ("reserved2", c_uint32)]


class he_lr_plan(ctypes.Structure):
    _fields_ = [("level_in", c_int32), ("level_out", c_int32)] + \
        [(n, c_double) for n in ("s1", "s_mask", "s_m", "s_a", "t", "s_z3", "s_b3", "s_c", "s_z1", "s_b1", "s_g")] + \
        [(n, c_int64) for n in ("k0", "k1", "k3", "kb1", "kw")] + [("s_z2", c_double), ("k2", c_int64)] + \
        [("s_gsum", c_double), ("layout", c_int32), ("reserved", c_int32)]


class he_infer_plan(ctypes.Structure):
    _fields_ = [("level_in", c_int32), ("level_out", c_int32)] + \
        [(n, c_double) for n in ("s_u", "s_u2", "s_h", "s_p")] + [(n, c_int64) for n in ("k3", "k2c", "k1", "k0c")]


class he_kernel_stat(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("launches", c_int32), ("ms", c_double), ("bytes", c_double),
                ("mm_fp64", c_double), ("mm_int", c_double)]


# kernel kinds of the trace (HE_K_*)
(K_NTT_FWD_COLS, K_NTT_FWD_ROWS, K_NTT_INV_ROWS, K_NTT_INV_COLS, K_NTT_ONE_LAUNCH, K_MD_CONV, K_MD_FINISH,
 K_MD_LAST, K_KS_COLS, K_KS_ROWS, K_MODUP, K_GIANT_FP64, K_GIANT_INT, K_ROT_INNER, K_BABY_SUM, K_TERMS_SUM,
 K_TENSOR, K_ELEMENTWISE, K_AUTOMORPH, K_GIANT_GATHER, K_OTHER, K_COUNT) = range(22)

LAYOUT_ROWS, LAYOUT_FEATURES = 0, 1  # HE_LAYOUT_ROWS / HE_LAYOUT_FEATURES
NOALLOC_SCRATCH_BYTES = 64 << 20  # HE_NOALLOC_SCRATCH_BYTES


_P = POINTER
_sig = {
    "he_strerror": (ctypes.c_char_p, [c_int]),
    "he_ctx_create": (c_int, [_P(he_params), c_void_p, c_void_p, c_void_p, c_void_p, _P(c_void_p)]),
    "he_ctx_destroy": (c_int, [c_void_p]),
    "he_ctx_set_stream": (c_int, [c_void_p, c_void_p]),
    "he_ctx_primes": (c_int, [c_void_p, _P(c_uint64), c_int]),
    "he_ctx_trim": (c_int, [c_void_p]),
    "he_ctx_set_ntt": (c_int, [c_void_p, c_int, c_int, c_int, c_int]),
    "he_params_primes": (c_int, [_P(he_params), _P(c_uint64), c_int]),
    "he_ct_bytes": (c_size_t, [c_void_p, c_int]),
    "he_pt_bytes": (c_size_t, [c_void_p, c_int]),
    "he_ct3_bytes": (c_size_t, [c_void_p, c_int]),
    "he_keys_bytes": (c_size_t, [c_void_p, c_int]),
    "he_keygen": (c_int, [c_void_p, c_uint64, _P(c_int32), c_int, c_void_p, c_size_t, _P(c_void_p)]),
    "he_keys_destroy": (c_int, [c_void_p]),
    "he_keys_download": (c_int, [c_void_p, c_void_p, c_int64, _P(c_uint64)]),
    "he_encode": (c_int, [c_void_p, _P(c_double), _P(c_double), c_int, c_double, _P(c_int64)]),
    "he_decode": (c_int, [c_void_p, _P(c_double), c_double, c_int, _P(c_double), _P(c_double)]),
    "he_pt_load": (c_int, [c_void_p, _P(c_int64), c_int, c_double, _P(he_pt)]),
    "he_encrypt": (c_int, [c_void_p, _P(he_pt), c_void_p, c_int, c_uint64, c_uint32, _P(he_ct)]),
    "he_decrypt": (c_int, [c_void_p, _P(he_ct), c_void_p, _P(c_uint64)]),
    "he_encrypt_seeded": (c_int, [c_void_p, _P(he_pt), c_void_p, c_uint64, c_uint32, _P(he_ct_seeded)]),
    "he_ct_expand": (c_int, [c_void_p, _P(he_ct_seeded), c_int, _P(he_ct)]),
    "he_lr_grad_step_seeded": (c_int, [c_void_p, _P(he_ct_seeded), c_int, _P(he_ct), _P(he_pt), _P(c_double), c_double,
                                       c_double, c_int, c_int, c_int, c_int, c_void_p, _P(he_ct), _P(he_ct)]),
    "he_lr_step_seeded_bytes": (c_size_t, [c_void_p, c_int, c_int, c_int, c_int]),
    "he_decrypt_decode": (c_int, [c_void_p, _P(he_ct), c_void_p, c_int, _P(c_double), _P(c_double)]),
    "he_ct_download": (c_int, [c_void_p, _P(he_ct), _P(c_uint64)]),
    "he_ct_upload": (c_int, [c_void_p, _P(c_uint64), c_int, c_double, _P(he_ct)]),
    "he_mul": (c_int, [c_void_p, _P(he_ct), _P(he_ct), _P(he_ct3)]),
    "he_relin": (c_int, [c_void_p, _P(he_ct3), c_void_p, _P(he_ct)]),
    "he_rescale": (c_int, [c_void_p, _P(he_ct), _P(he_ct)]),
    "he_rotate": (c_int, [c_void_p, _P(he_ct), c_int, c_void_p, _P(he_ct)]),
    "he_rotate_noalloc": (c_int, [c_void_p, _P(he_ct), c_int, c_void_p, _P(he_ct)]),
    "he_rotate_noalloc_bytes": (c_size_t, [c_void_p, c_int]),
    "he_add": (c_int, [c_void_p, _P(he_ct), _P(he_ct), _P(he_ct)]),
    "he_mul_int": (c_int, [c_void_p, _P(he_ct), c_int64, c_double, _P(he_ct)]),
    "he_mul_plain": (c_int, [c_void_p, _P(he_ct), _P(he_pt), _P(he_ct)]),
    "he_drop_level": (c_int, [c_void_p, _P(he_ct), c_int, _P(he_ct)]),
    "he_plan_lr_step": (c_int, [_P(c_uint64), c_int, c_int, c_double, c_double, _P(c_double), c_double, c_double,
                                c_int, _P(he_lr_plan)]),
    "he_lr_grad_step": (c_int, [c_void_p, _P(he_ct), c_int, _P(he_ct), _P(he_pt), _P(c_double), c_double, c_double,
                                c_int, c_int, c_int, _P(he_ct), c_int, _P(he_ct), c_void_p, c_int, _P(he_ct),
                                _P(he_ct)]),
    "he_lr_data_terms": (c_int, [c_void_p, _P(he_ct), c_int, c_int, c_double, _P(c_double), c_double, c_double, c_int,
                                 _P(he_ct)]),
    "he_rotate_many": (c_int, [c_void_p, _P(he_ct), c_int, _P(c_int32), c_int, c_void_p, _P(he_ct)]),
    "he_rotate_sum": (c_int, [c_void_p, _P(he_ct), c_int, _P(c_int32), c_int, c_void_p, _P(he_ct)]),
    "he_batch_mul_rotate": (c_int, [c_void_p, _P(he_ct), _P(he_ct), _P(c_int32), c_int, c_void_p, c_int,
                                    _P(he_ct)]),
    "he_batch_submit": (c_int, [c_void_p, _P(he_op), c_int, c_void_p, c_int]),
    "he_lr_grad_step_multi": (c_int, [c_void_p, _P(he_lr_request), c_int, c_int, c_int, c_int, c_void_p, c_int]),
    "he_lr_grad_step_multi_bytes": (ctypes.c_size_t, [c_void_p, c_int, c_int, c_int, c_int, c_int]),
    "he_batch_submit_bytes": (ctypes.c_size_t, [c_void_p, _P(he_op), c_int, c_int]),
    "he_lr_margins": (c_int, [c_void_p, _P(he_ct), c_int, _P(he_ct), c_int, c_int, c_int, c_void_p, c_int,
                              _P(he_ct)]),
    "he_lr_infer": (c_int, [c_void_p, _P(he_ct), c_int, _P(he_ct), c_int, c_int, c_int, _P(c_double), c_void_p,
                            c_int, _P(he_ct)]),
    "he_plan_lr_infer": (c_int, [_P(c_uint64), c_int, c_int, c_double, c_double, _P(c_double),
                                 _P(he_infer_plan)]),
    "he_lr_step_bytes": (c_size_t, [c_void_p, c_int, c_int, c_int, c_int, c_int]),
    "he_lr_margins_bytes": (c_size_t, [c_void_p, c_int, c_int, c_int]),
    "he_ntt": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int]),
    "he_valu_peak": (c_int, [c_void_p, c_int, c_int, _P(c_double)]),
    "he_ctx_trace": (c_int, [c_void_p, c_int]),
    "he_ctx_trace_read": (c_int, [c_void_p, _P(he_kernel_stat), c_int, _P(c_int)]),
    "he_kernel_kind_name": (ctypes.c_char_p, [c_int]),
}
for _n, (_r, _a) in _sig.items():
    _f = getattr(_lib, _n)
    _f.restype = _r
    _f.argtypes = _a

EXPORTS = sorted(_sig)


def _chk(st, where):
    if st != 0:
        raise HEError(st, where)


def _u64p(a):
    return a.ctypes.data_as(POINTER(c_uint64))


def _f64p(a):
    return a.ctypes.data_as(POINTER(c_double))


def _i64p(a):
    return a.ctypes.data_as(POINTER(c_int64))


def params_primes(log_n, n_q, n_special, alpha, log_delta):
    """Pure host: the prime chain selected by the parameters."""
    p = he_params(log_n, n_q, n_special, alpha, log_delta)
    out = np.zeros(n_q + n_special, dtype=np.uint64)
    _chk(_lib.he_params_primes(ctypes.byref(p), _u64p(out), n_q + n_special), "he_params_primes")
    return [int(v) for v in out]


def plan_lr_step(primes, n_q, level, s_z, s_w, coef, eta_over_n, w_decay=0.0, layout=LAYOUT_ROWS):
    """Pure host scale schedule (no device)."""
    q = np.ascontiguousarray(primes, dtype=np.uint64)
    cf = np.ascontiguousarray(coef, dtype=np.float64)
    out = he_lr_plan()
    _chk(_lib.he_plan_lr_step(_u64p(q), n_q, level, s_z, s_w, _f64p(cf), eta_over_n, w_decay, layout,
                              ctypes.byref(out)), "he_plan_lr_step")
    return {f[0]: getattr(out, f[0]) for f in he_lr_plan._fields_}


def plan_lr_infer(primes, n_q, level, s_z, s_w, coef):
    """Pure host schedule of he_lr_infer with the polynomial."""
    q = np.ascontiguousarray(primes, dtype=np.uint64)
    cf = np.ascontiguousarray(coef, dtype=np.float64)
    out = he_infer_plan()
    _chk(_lib.he_plan_lr_infer(_u64p(q), n_q, level, s_z, s_w, _f64p(cf), ctypes.byref(out)), "he_plan_lr_infer")
    return {f[0]: getattr(out, f[0]) for f in he_infer_plan._fields_}


class Ciphertext:
    """Device ciphertext (torch storage) + level and scale metadata."""

    def __init__(self, tensor, level, scale, offset=0):
        self.tensor = tensor
        self.level = level
        self.scale = scale
        self.offset = offset  # in uint64 elements

    @property
    def ptr(self):
        return self.tensor.data_ptr() + 8 * self.offset

    def struct(self):
        return he_ct(self.ptr, self.level, 0, self.scale)

    def update(self, s):
        self.level, self.scale = s.level, s.scale
        return self


Plaintext = Ciphertext


class SeededCiphertext:
    """Seeded ciphertext: its b component (torch storage) and the (seed,
    index) its uniform part is regenerated from."""

    def __init__(self, tensor, level, scale, seed, index, offset=0):
        self.tensor, self.level, self.scale, self.seed, self.index, self.offset = tensor, level, scale, seed, index, \
            offset

    def struct(self):
        return he_ct_seeded(self.tensor.data_ptr() + 8 * self.offset, self.level, 0, self.scale, self.seed,
                            self.index, 0)


# he_alloc_fn / he_free_fn: the library's device memory comes from torch
_ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_void_p, c_size_t)
_FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class TorchMemory:
    """Device memory provider of a context: every table and workspace the
    library holds is a torch uint8 tensor kept alive here until released."""

    def __init__(self, device):
        self.device = device
        self.live = {}
        self.alloc_fn = _ALLOC_FN(self._alloc)
        self.free_fn = _FREE_FN(self._free)

    def _alloc(self, user, nbytes):
        try:
            t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=self.device)
        except Exception:  # out of memory: the library returns HE_ENOMEM
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _free(self, user, ptr):
        if self.live is not None:
            self.live.pop(ptr, None)

    @property
    def bytes(self):
        """Device bytes the context holds now (tables and workspace)."""
        return sum(t.numel() for t in self.live.values())


class Keys:
    def __init__(self, ctx, buf, handle, rot_steps):
        self.ctx, self.buf, self.handle, self.rot_steps = ctx, buf, handle, list(rot_steps)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:  # _lib is None during interpreter teardown
            _lib.he_keys_destroy(self.handle)
            self.handle = None

    def download(self, which):
        c = self.ctx
        n = c.np * c.N if which == -2 else 2 * c.n_q * c.N if which == -5 else c.dnum * 2 * c.np * c.N
        out = np.zeros(n, dtype=np.uint64)
        _chk(_lib.he_keys_download(c.h, self.handle, which, _u64p(out)), "he_keys_download")
        return out


class Context:
    def __init__(self, log_n, n_q, n_special, alpha, log_delta, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device())
        p = he_params(log_n, n_q, n_special, alpha, log_delta)
        h = c_void_p()
        s = torch.cuda.current_stream().cuda_stream if stream is None else stream
        self.mem = TorchMemory(self.device)
        _chk(_lib.he_ctx_create(ctypes.byref(p), ctypes.cast(self.mem.alloc_fn, c_void_p),
                                ctypes.cast(self.mem.free_fn, c_void_p), None, c_void_p(s), ctypes.byref(h)),
             "he_ctx_create")
        self.h = h
        self.log_n, self.n_q, self.n_special, self.alpha, self.log_delta = log_n, n_q, n_special, alpha, log_delta
        self.N = 1 << log_n
        self.S = self.N // 2
        self.np = n_q + n_special
        self.dnum = (n_q + alpha - 1) // alpha
        q = np.zeros(self.np, dtype=np.uint64)
        _chk(_lib.he_ctx_primes(self.h, _u64p(q), self.np), "he_ctx_primes")
        self.primes = [int(v) for v in q]
        from . import autotune  # the measured NTT launch shape for this ring degree, if tuned
        self.ntt_tuned = autotune.apply(self)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.he_ctx_destroy(self.h)
            self.h = None

    @property
    def delta(self):
        return float(2 ** self.log_delta)

    # ------------------------------------------------------------ memory
    def _alloc(self, n_u64):
        return self.torch.empty(int(n_u64), dtype=self.torch.int64, device=self.device)

    def ct_empty(self, level):
        return Ciphertext(self._alloc(2 * (level + 1) * self.N), level, 0.0)

    def ct3_empty(self, level):
        return Ciphertext(self._alloc(3 * (level + 1) * self.N), level, 0.0)

    def pt_empty(self, level):
        return Ciphertext(self._alloc((level + 1) * self.N), level, 0.0)

    def ct_block(self, count, level):
        """count ciphertexts at one level in one allocation (uniform stride)."""
        per = 2 * (level + 1) * self.N
        t = self._alloc(per * count)
        return [Ciphertext(t, level, 0.0, offset=i * per) for i in range(count)]

    def set_ntt(self, persistent=1, wg_per_xcd=64, lag=2, min_limbs=1):
        """he_ctx_set_ntt: launch shape of the plain NTTs (bit-identical results)."""
        _chk(_lib.he_ctx_set_ntt(self.h, int(persistent), int(wg_per_xcd), int(lag), int(min_limbs)),
             "he_ctx_set_ntt")

    def trim(self):
        _chk(_lib.he_ctx_trim(self.h), "he_ctx_trim")

    # ------------------------------------------------------------ keys / encoding
    def keygen(self, seed, rot_steps=()):
        steps = np.ascontiguousarray(list(rot_steps), dtype=np.int32)
        nbytes = _lib.he_keys_bytes(self.h, len(steps))
        buf = self._alloc((nbytes + 7) // 8)
        h = c_void_p()
        _chk(_lib.he_keygen(self.h, seed, steps.ctypes.data_as(POINTER(c_int32)), len(steps), c_void_p(buf.data_ptr()),
                            nbytes, ctypes.byref(h)), "he_keygen")
        return Keys(self, buf, h, rot_steps)

    def encode(self, values, scale):
        v = np.asarray(values)
        re = np.ascontiguousarray(v.real, dtype=np.float64)
        im = np.ascontiguousarray(v.imag, dtype=np.float64) if np.iscomplexobj(v) else None
        out = np.zeros(self.N, dtype=np.int64)
        _chk(_lib.he_encode(self.h, _f64p(re), _f64p(im) if im is not None else None, re.shape[0], scale,
                            _i64p(out)), "he_encode")
        return out

    def decode(self, coeffs, scale, n=None):
        m = np.ascontiguousarray(coeffs, dtype=np.float64)
        n = self.S if n is None else n
        re, im = np.zeros(n), np.zeros(n)
        _chk(_lib.he_decode(self.h, _f64p(m), scale, n, _f64p(re), _f64p(im)), "he_decode")
        return re + 1j * im

    def pt_load(self, coeffs, level, scale, out=None):
        out = out or self.pt_empty(level)
        m = np.ascontiguousarray(coeffs, dtype=np.int64)
        s = out.struct()
        _chk(_lib.he_pt_load(self.h, _i64p(m), level, scale, ctypes.byref(s)), "he_pt_load")
        return out.update(s)

    # ------------------------------------------------------------ encryption
    def encrypt(self, pt, keys, seed, index, out=None, use_sk=True):
        """Secret-key (use_sk, Alg. 2's server) or public-key (Alg. 1's worker) encryption."""
        out = out or self.ct_empty(pt.level)
        p, s = pt.struct(), out.struct()
        _chk(_lib.he_encrypt(self.h, ctypes.byref(p), keys.handle, 1 if use_sk else 0, seed, index, ctypes.byref(s)),
             "he_encrypt")
        return out.update(s)

    def seeded_block(self, count, level):
        """count seeded ciphertexts' b-parts at one level in one allocation."""
        per = (level + 1) * self.N
        t = self._alloc(per * count)
        return [SeededCiphertext(t, level, 0.0, 0, 0, offset=i * per) for i in range(count)]

    def encrypt_seeded(self, pt, keys, seed, index, out=None):
        """he_encrypt_seeded: b only; the uniform part is (seed, index)."""
        out = out or self.seeded_block(1, pt.level)[0]
        p, s = pt.struct(), out.struct()
        _chk(_lib.he_encrypt_seeded(self.h, ctypes.byref(p), keys.handle, seed, index, ctypes.byref(s)),
             "he_encrypt_seeded")
        out.level, out.scale, out.seed, out.index = s.level, s.scale, s.seed, s.index
        return out

    def expand(self, xs, outs=None):
        outs = outs or [self.ct_empty(x.level) for x in xs]
        xa = (he_ct_seeded * len(xs))(*[x.struct() for x in xs])
        oa = (he_ct * len(xs))(*[o.struct() for o in outs])
        _chk(_lib.he_ct_expand(self.h, xa, len(xs), oa), "he_ct_expand")
        for o, s_ in zip(outs, oa):
            o.update(s_)
        return outs

    def lr_grad_step_seeded(self, Z, W, mask, coef, eta_over_n, cols, rows, keys, chunk, W_out=None, G_out=None,
                            want_g=True, w_decay=0.0, layout=LAYOUT_ROWS):
        """he_lr_grad_step_seeded: the step over seeded blocks, `chunk` blocks at a time."""
        za = Z if isinstance(Z, ctypes.Array) else (he_ct_seeded * len(Z))(*[z.struct() for z in Z])
        w, m = W.struct(), mask.struct()
        lo = W.level - 4
        W_out = W_out or self.ct_empty(lo)
        if want_g:
            G_out = G_out or self.ct_empty(lo)
        wo = W_out.struct()
        go = G_out.struct() if want_g else None
        cf = np.ascontiguousarray(coef, dtype=np.float64)
        _chk(_lib.he_lr_grad_step_seeded(self.h, za, len(za), ctypes.byref(w), ctypes.byref(m), _f64p(cf),
                                         eta_over_n, w_decay, cols, rows, layout, chunk, keys.handle,
                                         ctypes.byref(wo), ctypes.byref(go) if go is not None else None),
             "he_lr_grad_step_seeded")
        W_out.update(wo)
        if want_g:
            G_out.update(go)
        return W_out, (G_out if want_g else None)

    def step_seeded_bytes(self, level, data_level, chunk, layout=LAYOUT_ROWS):
        return int(_lib.he_lr_step_seeded_bytes(self.h, level, data_level, chunk, layout))

    def decrypt(self, ct, keys):
        out = np.zeros((ct.level + 1, self.N), dtype=np.uint64)
        s = ct.struct()
        _chk(_lib.he_decrypt(self.h, ctypes.byref(s), keys.handle, _u64p(out)), "he_decrypt")
        return out

    def decrypt_decode(self, ct, keys, n=None):
        n = self.S if n is None else n
        re, im = np.zeros(n), np.zeros(n)
        s = ct.struct()
        _chk(_lib.he_decrypt_decode(self.h, ctypes.byref(s), keys.handle, n, _f64p(re), _f64p(im)),
             "he_decrypt_decode")
        return re + 1j * im

    def download(self, ct):
        out = np.zeros((2, ct.level + 1, self.N), dtype=np.uint64)
        s = ct.struct()
        _chk(_lib.he_ct_download(self.h, ctypes.byref(s), _u64p(out)), "he_ct_download")
        return out

    def upload(self, arr, level, scale, out=None):
        out = out or self.ct_empty(level)
        a = np.ascontiguousarray(arr, dtype=np.uint64)
        assert a.shape == (2, level + 1, self.N)
        s = out.struct()
        _chk(_lib.he_ct_upload(self.h, _u64p(a), level, scale, ctypes.byref(s)), "he_ct_upload")
        return out.update(s)

    # ------------------------------------------------------------ operations
    def mul(self, x, y, out=None):
        out = out or self.ct3_empty(x.level)
        a, b, o = x.struct(), y.struct(), out.struct()
        _chk(_lib.he_mul(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(o)), "he_mul")
        return out.update(o)

    def relin(self, d, keys, out=None):
        out = out or self.ct_empty(d.level)
        a, o = d.struct(), out.struct()
        _chk(_lib.he_relin(self.h, ctypes.byref(a), keys.handle, ctypes.byref(o)), "he_relin")
        return out.update(o)

    def rescale(self, x, out=None):
        out = out or self.ct_empty(max(x.level - 1, 0))
        a, o = x.struct(), out.struct()
        _chk(_lib.he_rescale(self.h, ctypes.byref(a), ctypes.byref(o)), "he_rescale")
        return out.update(o)

    def rotate(self, x, steps, keys, out=None):
        out = out or self.ct_empty(x.level)
        a, o = x.struct(), out.struct()
        _chk(_lib.he_rotate(self.h, ctypes.byref(a), steps, keys.handle, ctypes.byref(o)), "he_rotate")
        return out.update(o)

    def _noalloc_bytes(self, level):
        return int(_lib.he_rotate_noalloc_bytes(self.h, level))

    def rotate_noalloc(self, x, steps, keys, out):
        """he_rotate_noalloc: he_rotate with no device allocation; out is the
        caller's (a ciphertext at x's level)."""
        a, o = x.struct(), out.struct()
        _chk(_lib.he_rotate_noalloc(self.h, ctypes.byref(a), steps, keys.handle, ctypes.byref(o)), "he_rotate_noalloc")
        return out.update(o)

    def add(self, x, y, out=None):
        out = out or self.ct_empty(x.level)
        a, b, o = x.struct(), y.struct(), out.struct()
        _chk(_lib.he_add(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(o)), "he_add")
        return out.update(o)

    def mul_int(self, x, k, out_scale, out=None):
        out = out or self.ct_empty(x.level)
        a, o = x.struct(), out.struct()
        _chk(_lib.he_mul_int(self.h, ctypes.byref(a), int(k), out_scale, ctypes.byref(o)), "he_mul_int")
        return out.update(o)

    def mul_plain(self, x, pt, out=None):
        out = out or self.ct_empty(x.level)
        a, p, o = x.struct(), pt.struct(), out.struct()
        _chk(_lib.he_mul_plain(self.h, ctypes.byref(a), ctypes.byref(p), ctypes.byref(o)), "he_mul_plain")
        return out.update(o)

    def drop_level(self, x, level, out=None):
        out = out or self.ct_empty(level)
        a, o = x.struct(), out.struct()
        _chk(_lib.he_drop_level(self.h, ctypes.byref(a), level, ctypes.byref(o)), "he_drop_level")
        return out.update(o)

    def plan_lr_step(self, level, s_z, s_w, coef, eta_over_n, w_decay=0.0, layout=LAYOUT_ROWS):
        return plan_lr_step(self.primes, self.n_q, level, s_z, s_w, coef, eta_over_n, w_decay, layout)

    def lr_grad_step(self, Z, W, mask, coef, eta_over_n, cols, rows, keys, mode=1, W_out=None, G_out=None,
                     want_g=True, w_decay=0.0, layout=LAYOUT_ROWS, Zrot=None, n_baby=1, Zk=None):
        """One encrypted gradient step (he_lr_grad_step).  Z: list of block
        ciphertexts sharing one allocation (ct_block), packed in `layout`;
        with n_baby > 1: Zrot = rotate_data(Z, baby_unit(layout, rows), n_baby);
        Zk: lr_data_terms for this W's level and scale, or None.  Z, Zrot and Zk
        may also be ct_array()s built once (callers stepping many times skip
        rebuilding the argument arrays).  Returns (W', g)."""
        zs = ct_array(Z)
        zr = ct_array(Zrot) if Zrot else None
        zk = ct_array(Zk) if Zk else None
        w, m = W.struct(), mask.struct()
        lo = max(W.level - 4, 0)
        W_out = W_out or self.ct_empty(lo)
        if want_g:
            G_out = G_out or self.ct_empty(lo)
        wo = W_out.struct()
        go = G_out.struct() if want_g else None
        cf = np.ascontiguousarray(coef, dtype=np.float64)
        _chk(_lib.he_lr_grad_step(self.h, zs, len(Z), ctypes.byref(w), ctypes.byref(m), _f64p(cf), eta_over_n,
                                  w_decay, cols, rows, layout, zr, n_baby, zk, keys.handle, mode, ctypes.byref(wo),
                                  ctypes.byref(go) if go is not None else None), "he_lr_grad_step")
        W_out.update(wo)
        if want_g:
            G_out.update(go)
        return W_out, (G_out if want_g else None)

    def lr_grad_step_multi(self, requests, cols, rows, keys, mode=1, layout=LAYOUT_ROWS):
        """he_lr_grad_step_multi over requests = [dict(Z=, W=, mask=, coef=, eta_over_n=, w_decay=0.0,
        W_out=None, G_out=None)] (outputs allocated when None; G_out=False: no g); returns [(W', g)]."""
        n = len(requests)
        arr = (he_lr_request * n)()
        keep = []
        outs = []
        for a, rq in zip(arr, requests):
            zs = ct_array(rq["Z"])
            w, m = rq["W"].struct(), rq["mask"].struct()
            cf = np.ascontiguousarray(rq["coef"], dtype=np.float64)
            lo = max(rq["W"].level - 4, 0)
            Wo = rq.get("W_out") or self.ct_empty(lo)
            Go = rq.get("G_out")
            Go = None if Go is False else (Go or self.ct_empty(lo))
            wo = Wo.struct()
            go = Go.struct() if Go is not None else None
            keep += [zs, w, m, cf, wo, go]
            a.Z = ctypes.cast(zs, POINTER(he_ct))
            a.n_blocks = len(rq["Z"])
            a.W = ctypes.pointer(w)
            a.mask = ctypes.pointer(m)
            a.coef = _f64p(cf)
            a.eta_over_n = rq["eta_over_n"]
            a.w_decay = rq.get("w_decay", 0.0)
            a.W_out = ctypes.pointer(wo)
            a.G_out = ctypes.pointer(go) if go is not None else None
            outs.append((Wo, wo, Go, go))
        _chk(_lib.he_lr_grad_step_multi(self.h, arr, n, cols, rows, layout, keys.handle, mode),
             "he_lr_grad_step_multi")
        res = []
        for Wo, wo, Go, go in outs:
            Wo.update(wo)
            if Go is not None:
                Go.update(go)
            res.append((Wo, Go))
        return res

    def step_multi_bytes(self, level, max_blocks, n_req, layout=LAYOUT_ROWS, mode=1):
        return int(_lib.he_lr_grad_step_multi_bytes(self.h, level, max_blocks, n_req, layout, mode))

    def lr_data_terms(self, Z, w_level, w_scale, coef, eta_over_n, w_decay=0.0, layout=LAYOUT_ROWS):
        """he_lr_data_terms: RS(k3 Z), RS(k1 Z) (and RS(k2 Z) when coef[2] != 0)
        for weights at w_level with scale w_scale, one ct_block per group;
        returns the list in the order he_lr_grad_step's Zk takes."""
        fm = layout == LAYOUT_FEATURES
        l3, l1 = (w_level - 1, w_level - 2) if fm else (w_level - 2, w_level - 3)
        groups = [self.ct_block(len(Z), l3), self.ct_block(len(Z), l1)]
        if coef[2] != 0:
            groups.append(self.ct_block(len(Z), l1))
        out = [o for g in groups for o in g]
        oa = (he_ct * len(out))(*[o.struct() for o in out])
        cf = np.ascontiguousarray(coef, dtype=np.float64)
        _chk(_lib.he_lr_data_terms(self.h, ct_array(Z), len(Z), w_level, w_scale, _f64p(cf), eta_over_n, w_decay,
                                   layout, oa), "he_lr_data_terms")
        for o, s_ in zip(out, oa):
            o.update(s_)
        return out

    def lr_margins(self, Z, W, cols, rows, keys, mode=1, out=None, layout=LAYOUT_ROWS):
        """he_lr_margins: per block u = RS(relin(Z_b (x) W)) + the margin sum.
        out: list of len(Z) ciphertexts at W.level - 1 with one stride
        (ct_block); allocated when None."""
        out = out or self.ct_block(len(Z), W.level - 1)
        zs = (he_ct * len(Z))(*[z.struct() for z in Z])
        os_ = (he_ct * len(out))(*[o.struct() for o in out])
        w = W.struct()
        _chk(_lib.he_lr_margins(self.h, zs, len(Z), ctypes.byref(w), cols, rows, layout, keys.handle, mode, os_),
             "he_lr_margins")
        for o, s_ in zip(out, os_):
            o.update(s_)
        return out

    def lr_infer(self, Z, W, cols, rows, keys, coef=None, mode=1, out=None, layout=LAYOUT_ROWS):
        """he_lr_infer: the margins (coef None) or p(margins) slot by slot, per
        block; out: list of len(Z) ciphertexts with one stride (ct_block) at
        W.level - 1 (margins) or W.level - 3 (polynomial); allocated when None."""
        lo = W.level - 1 if coef is None else W.level - 3
        out = out or self.ct_block(len(Z), lo)
        zs = ct_array(Z)
        os_ = (he_ct * len(out))(*[o.struct() for o in out])
        w = W.struct()
        cf = np.ascontiguousarray(coef, dtype=np.float64) if coef is not None else None
        _chk(_lib.he_lr_infer(self.h, zs, len(Z), ctypes.byref(w), cols, rows, layout,
                              _f64p(cf) if cf is not None else None, keys.handle, mode, os_), "he_lr_infer")
        for o, s_ in zip(out, os_):
            o.update(s_)
        return out

    def step_bytes(self, level, n_blocks, layout=LAYOUT_ROWS, mode=1, n_baby=1):
        return int(_lib.he_lr_step_bytes(self.h, level, n_blocks, layout, n_baby, mode))

    def rotate_many(self, xs, steps, keys, outs=None):
        """he_rotate_many: outs[i * len(steps) + s] = Rot(xs[i], steps[s]);
        outs allocated as one block when None."""
        m = len(xs) * len(steps)
        outs = outs or self.ct_block(m, xs[0].level)
        xa = (he_ct * len(xs))(*[x.struct() for x in xs])
        oa = (he_ct * m)(*[o.struct() for o in outs])
        st = np.ascontiguousarray(steps, dtype=np.int32)
        _chk(_lib.he_rotate_many(self.h, xa, len(xs), st.ctypes.data_as(POINTER(c_int32)), len(steps), keys.handle,
                                 oa), "he_rotate_many")
        for o, s_ in zip(outs, oa):
            o.update(s_)
        return outs

    def rotate_sum(self, xs, steps, keys, outs=None):
        """he_rotate_sum: outs[i] = xs[i] + sum_s Rot(xs[i], steps[s]), one
        hoisted key switch each; outs allocated as one block when None."""
        outs = outs or self.ct_block(len(xs), xs[0].level)
        xa = (he_ct * len(xs))(*[x.struct() for x in xs])
        oa = (he_ct * len(xs))(*[o.struct() for o in outs])
        st = np.ascontiguousarray(steps, dtype=np.int32)
        _chk(_lib.he_rotate_sum(self.h, xa, len(xs), st.ctypes.data_as(POINTER(c_int32)), len(steps), keys.handle,
                                oa), "he_rotate_sum")
        for o, s_ in zip(outs, oa):
            o.update(s_)
        return outs

    def rotate_data(self, Z, unit, n_baby, keys):
        """The baby-step copies of a shard for lr_grad_step: Rot(Z[b], j unit)
        for j = 1 .. n_baby - 1, block by block (unit = baby_unit(layout,
        rows))."""
        if n_baby <= 1:
            return None
        return self.rotate_many(Z, [j * unit for j in range(1, n_baby)], keys)

    def margins_bytes(self, level, n_blocks, mode=1):
        return int(_lib.he_lr_margins_bytes(self.h, level, n_blocks, mode))

    def batch_mul_rotate(self, xs, ys, steps, keys, mode=1, outs=None):
        """he_batch_mul_rotate: out[i] = Rot(RS(relin(x[i] (x) y[i])), steps[i])."""
        n = len(xs)
        outs = outs or [self.ct_empty(x.level - 1) for x in xs]
        xa = (he_ct * n)(*[x.struct() for x in xs])
        ya = (he_ct * n)(*[y.struct() for y in ys])
        oa = (he_ct * n)(*[o.struct() for o in outs])
        st = np.ascontiguousarray(steps, dtype=np.int32)
        _chk(_lib.he_batch_mul_rotate(self.h, xa, ya, st.ctypes.data_as(POINTER(c_int32)), n, keys.handle, mode, oa),
             "he_batch_mul_rotate")
        for o, s_ in zip(outs, oa):
            o.update(s_)
        return outs

    @staticmethod
    def op_out_level(op, x):
        return x.level - 1 if op in (OP_MUL, OP_MUL_ROTATE, OP_RESCALE) else x.level

    def op_array(self, ops):
        """he_op array of [(op, steps, x, y, out)] (y None where unused; out
        allocated at the op's output level when None); returns (array, outs)."""
        outs = [o if o is not None else self.ct_empty(self.op_out_level(op, x)) for op, _, x, _, o in ops]
        arr = (he_op * len(ops))()
        for a, (op, steps, x, y, _), o in zip(arr, ops, outs):
            a.op, a.steps, a.x, a.out = op, int(steps), x.struct(), o.struct()
            if y is not None:
                a.y = y.struct()
        return arr, outs

    def batch_submit(self, ops, keys, mode=1):
        """he_batch_submit over [(op, steps, x, y, out)]; returns the outs."""
        arr, outs = self.op_array(ops)
        _chk(_lib.he_batch_submit(self.h, arr, len(ops), keys.handle, mode), "he_batch_submit")
        for o, a in zip(outs, arr):
            o.update(a.out)
        return outs

    def batch_submit_bytes(self, ops, mode=1):
        arr, _ = self.op_array(ops)
        return int(_lib.he_batch_submit_bytes(self.h, arr, len(ops), mode))

    def valu_peak(self, prime_idx, fp64=True):
        """he_valu_peak: measured butterflies per second of the NTT's butterfly."""
        v = c_double()
        _chk(_lib.he_valu_peak(self.h, prime_idx, 1 if fp64 else 0, ctypes.byref(v)), "he_valu_peak")
        return v.value

    def trace(self, on=True):
        """he_ctx_trace: record every launch (outside capture) with HIP events."""
        _chk(_lib.he_ctx_trace(self.h, 1 if on else 0), "he_ctx_trace")

    def trace_read(self):
        """he_ctx_trace_read: per kernel kind, launches, ms, algorithmic bytes
        and modular products since tracing was switched on (clears them)."""
        arr = (he_kernel_stat * K_COUNT)()
        n = c_int()
        _chk(_lib.he_ctx_trace_read(self.h, arr, K_COUNT, ctypes.byref(n)), "he_ctx_trace_read")
        return [dict(kind=a.kind, name=_lib.he_kernel_kind_name(a.kind).decode(), launches=a.launches, ms=a.ms,
                     bytes=a.bytes, mm_fp64=a.mm_fp64, mm_int=a.mm_int) for a in arr[:n.value]]

    def ntt(self, tensor, n_limbs, prime_idx0, period, direction):
        _chk(_lib.he_ntt(self.h, c_void_p(tensor.data_ptr()), n_limbs, prime_idx0, period, direction), "he_ntt")


# ---------------------------------------------------------------- packing (data layout of the step)
def pack_blocks(X, y, S, layout=LAYOUT_ROWS):
    """Blocks of Z = y (.) X; c = next power of two >= d, r = S / c.
    Row-major: slot i*c + j of block b holds y_{b r + i} x_{b r + i, j};
    feature-major: slot j*r + i holds it."""
    n, d = X.shape
    c = 1
    while c < d:
        c *= 2
    r = S // c
    nb = -(-n // r)
    Z = np.zeros((nb * r, c))
    Z[:n, :d] = y[:, None] * X
    Z = Z.reshape(nb, r, c)
    if layout == LAYOUT_FEATURES:
        Z = Z.transpose(0, 2, 1)
    return np.ascontiguousarray(Z).reshape(nb, S), c, r


def pack_weights(w, S, c, layout=LAYOUT_ROWS):
    """w in every row (row-major) or w_j over feature block j (feature-major)."""
    row = np.zeros(c)
    row[: len(w)] = w
    return np.repeat(row, S // c) if layout == LAYOUT_FEATURES else np.tile(row, S // c)


def unpack_weights(slots, c, d, layout=LAYOUT_ROWS):
    """w from the first row (row-major) or the first slot of each feature block."""
    v = np.asarray(slots)
    if layout == LAYOUT_FEATURES:
        return v.reshape(c, -1)[:d, 0]
    return v.reshape(-1, c)[0, :d]


def column0_mask(S, c):
    m = np.zeros(S)
    m[::c] = 1.0
    return m


def step_mask(S, c, layout=LAYOUT_ROWS):
    """The step's mask: column 0 of every row (row-major, applied to the
    margins) or slot 0 of every feature block (feature-major, applied to the
    gradient)."""
    m = np.zeros(S)
    m[:: (S // c) if layout == LAYOUT_FEATURES else c] = 1.0
    return m


def mask_level(level, layout=LAYOUT_ROWS):
    """Level of the step's mask plaintext for weights at `level`."""
    return level - 3 if layout == LAYOUT_FEATURES else level - 1


def baby_unit(layout, rows):
    """Rotation unit of the margin sum's baby steps: a feature block (rows
    slots) feature-major, one slot row-major."""
    return rows if layout == LAYOUT_FEATURES else 1


def ct_array(cts):
    """he_ct array argument for a list of ciphertexts (returned unchanged when
    it already is one)."""
    if isinstance(cts, ctypes.Array):
        return cts
    return (he_ct * len(cts))(*[c.struct() for c in cts])


GIANT_MAX = 16  # most giant steps a hoisted feature-major giant sum takes


def giant_hoisted(layout, c, n_baby):
    """Feature-major margins with 1 < n_baby < c and c / n_baby <= GIANT_MAX
    take their giant steps g n_baby r as one hoisted sum."""
    return layout == LAYOUT_FEATURES and 1 < n_baby < c and c // n_baby <= GIANT_MAX


def slot_sum_groups(count):
    """The rotation-index groups of a slot sum over count = 2^k multiples of
    a unit (he_lr_grad_step's and he_lr_margins' sums; one hoisted sum per
    group, its rotations scaled by the unit): the k bits of the
    index in ceil(k / 3) groups, sizes as even as possible (the smaller ones
    first), low bits first; a group of s bits from bit b0 holds the
    rotations j 2^b0, j = 1 .. 2^s - 1."""
    k = int(count).bit_length() - 1
    if k <= 0:
        return []
    ng = (k + 2) // 3
    q, rem = divmod(k, ng)
    out, b0 = [], 0
    for i in range(ng):
        size = q + (1 if i >= ng - rem else 0)
        out.append([j << b0 for j in range(1, 1 << size)])
        b0 += size
    return out


def rotation_steps(c, r, layout=LAYOUT_ROWS, n_baby=1):
    """Rotation keys the step needs (with n_baby baby steps also j u, j < n_baby,
    u = baby_unit(layout, r); with a hoisted giant sum also g n_baby r,
    g < c / n_baby).  Row-major: the baby steps j < n_baby, n_baby t for
    every t of slot_sum_groups(c / n_baby) (the column sum), -t for every t
    of slot_sum_groups(c) (the replication) and c t for every t of
    slot_sum_groups(r) (the row sum); feature-major: without a hoisted giant
    sum n_baby r t for every t of slot_sum_groups(c / n_baby) (the margin
    sum), and +-t for every t of slot_sum_groups(r) (the sample sum and the
    replication).  With n_baby = 1 the set also serves he_lr_margins and
    he_lr_infer in the same layout."""
    mu = baby_unit(layout, r)
    nb = max(n_baby, 1)
    if layout == LAYOUT_FEATURES:
        out = {j * mu for j in range(1, nb)}
        if giant_hoisted(layout, c, nb):
            out |= {g * nb * r for g in range(1, c // nb)}
        else:
            out |= {nb * r * t for grp in slot_sum_groups(c // nb) for t in grp}
        out |= {s * t for grp in slot_sum_groups(r) for t in grp for s in (1, -1)}
        return sorted(out)
    out = set(range(1, nb))
    out |= {nb * t for grp in slot_sum_groups(c // nb) for t in grp}
    out |= {-t for grp in slot_sum_groups(c) for t in grp}
    out |= {c * t for grp in slot_sum_groups(r) for t in grp}
    return sorted(out)
