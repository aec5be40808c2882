"""Python binding of libpfx.so (ctypes): the C-ABI of include/pfx.h under the
same names, with argument marshalling only.  Every step of the evaluation
runs in the library's HIP kernels; nothing here computes on the data.

Importing this module loads the in-tree ``libpfx.so`` and raises
``ImportError`` if it is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libpfx.so is not built at {LIB_PATH}; run __graft_entry__.build()")

_lib = ctypes.CDLL(LIB_PATH)

PFX_OK, PFX_EINVAL, PFX_EPARAM, PFX_ELEVEL, PFX_ESCALE = 0, -1, -2, -3, -4
PFX_ENOKEY, PFX_ENOMEM, PFX_EBUSY, PFX_EDEVICE = -5, -6, -7, -8
MAX_PRIMES = 64


class PfxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pfx error {status}: {msg}")
        self.status = status


class pfx_params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_q", ctypes.c_uint32),
                ("q_bits", ctypes.c_uint32 * MAX_PRIMES), ("n_p", ctypes.c_uint32),
                ("p_bits", ctypes.c_uint32 * MAX_PRIMES), ("alpha", ctypes.c_uint32),
                ("mod_log2", ctypes.c_uint32)]


class pfx_pass_tuning(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("row_wg256", ctypes.c_uint32), ("col_wg256", ctypes.c_uint32),
                ("widen_wg", ctypes.c_uint32), ("min_col", ctypes.c_uint32), ("min_col_special", ctypes.c_uint32),
                ("rs_widen_wg", ctypes.c_uint32), ("ks_fuse", ctypes.c_uint32), ("ks_batch", ctypes.c_uint32),
                ("ks_modup_batch", ctypes.c_uint32)]


class pfx_op(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("dst", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32),
                ("k", ctypes.c_int64), ("value", ctypes.c_double)]


OP_COPY, OP_ADD, OP_SUB, OP_MUL_PLAIN, OP_ADD_PLAIN, OP_MUL_INT, OP_MUL_RELIN = 0, 1, 2, 3, 4, 5, 6
OP_RESCALE, OP_ADD_CONST, OP_MUL_CONST, OP_SCALE_MUL, OP_ROTATE, OP_ROTATE_SUM = 7, 8, 9, 10, 11, 12
OP_LANE, OP_MUL, OP_RELIN, OP_MUL_ACC, OP_MUL_PLAIN_ACC, OP_MUL_INT_ACC, OP_DROP = 13, 14, 15, 16, 17, 18, 19
OP_MONO, OP_INV_N, OP_GALOIS, OP_MUL_CONST_TO, OP_MUL_CONST_LIKE = 20, 21, 22, 23, 24


class pfx_info(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_limbs", ctypes.c_uint32),
                ("degree", ctypes.c_uint32), ("scale", ctypes.c_double)]


class pfx_request(ctypes.Structure):
    _fields_ = [("ops", ctypes.POINTER(pfx_op)), ("n_ops", ctypes.c_size_t), ("n_regs", ctypes.c_size_t),
                ("n_inputs", ctypes.c_size_t), ("inputs", ctypes.POINTER(ctypes.c_void_p)),
                ("pts", ctypes.POINTER(ctypes.c_void_p)), ("n_pts", ctypes.c_size_t),
                ("out_reg", ctypes.c_int32), ("out", ctypes.c_void_p),
                ("reg_degree", ctypes.POINTER(ctypes.c_uint8))]


class pfx_request_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slot", ctypes.c_int32), ("footprint", ctypes.c_size_t),
                ("queued_s", ctypes.c_double), ("latency_s", ctypes.c_double), ("error", ctypes.c_char * 160)]


class pfx_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "queued", "running")] + \
               [(n, ctypes.c_size_t) for n in ("budget", "scratch_bytes", "arena_bytes", "bytes_in_use",
                                               "peak_bytes")] + \
               [("slots", ctypes.c_uint32), ("peak_running", ctypes.c_uint32)]


_vp = ctypes.c_void_p
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i8p = ctypes.POINTER(ctypes.c_int8)
_f64p = ctypes.POINTER(ctypes.c_double)
_u32, _i32, _sz, _i64 = ctypes.c_uint32, ctypes.c_int32, ctypes.c_size_t, ctypes.c_int64
_PP = ctypes.POINTER(pfx_params)
_IP = ctypes.POINTER(pfx_info)
_VPP = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "pfx_status_str": (ctypes.c_char_p, [_i32]),
    "pfx_last_error": (ctypes.c_char_p, []),
    "pfx_params_primes": (_i32, [_PP, _u64p, _u64p, _u64p]),
    "pfx_encode_words": (_i32, [_PP, _f64p, _f64p, _sz, _u32, ctypes.c_double, _u64p]),
    "pfx_decode_words": (_i32, [_PP, _u64p, _u32, ctypes.c_double, _f64p, _f64p, _sz]),
    "pfx_ctx_create": (_i32, [_PP, ctypes.c_int, _VPP]),
    "pfx_ctx_destroy": (None, [_vp]),
    "pfx_ctx_moduli": (_i32, [_vp, _u64p, _u64p, _u64p]),
    "pfx_sync": (_i32, [_vp, _vp]),
    "pfx_sk_create": (_i32, [_vp, _i8p, _VPP]),
    "pfx_sk_destroy": (None, [_vp]),
    "pfx_swk_create": (_i32, [_vp, _vp, _u32, _u64p, _i64p, _VPP]),
    "pfx_swk_export": (_i32, [_vp, _vp, _u64p, _sz]),
    "pfx_swk_galois": (_u32, [_vp]),
    "pfx_swk_import": (_i32, [_vp, _u32, _u64p, _sz, _VPP]),
    "pfx_sk_export": (_i32, [_vp, _vp, _sz]),
    "pfx_keygen_secret": (_i32, [_vp, _vp, _i32, _VPP]),
    "pfx_keygen_relin": (_i32, [_vp, _vp, _vp, _VPP]),
    "pfx_keygen_galois": (_i32, [_vp, _vp, _vp, _sz, ctypes.c_int, _vp, _VPP]),
    "pfx_encrypt_seeded": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "pfx_shake256": (_i32, [_vp, _sz, _vp, _sz]),
    "pfx_sample_uniform": (_i32, [_vp, _u32, _u32, _u32, ctypes.c_uint64, _sz, _u64p]),
    "pfx_sample_secret": (_i32, [_vp, _sz, _i32, _vp]),
    "pfx_sample_gaussian": (_i32, [_vp, _u32, _u32, _sz, _i64p]),
    "pfx_swk_destroy": (None, [_vp]),
    "pfx_encode": (_i32, [_vp, _f64p, _f64p, _sz, _u32, ctypes.c_double, _VPP]),
    "pfx_decode": (_i32, [_vp, _vp, _f64p, _f64p, _sz]),
    "pfx_pt_import": (_i32, [_vp, _u64p, _u32, ctypes.c_double, _VPP]),
    "pfx_encrypt": (_i32, [_vp, _vp, _vp, _u64p, _i64p, _vp, _vp]),
    "pfx_decrypt": (_i32, [_vp, _vp, _vp, _VPP, _vp]),
    "pfx_ct_create": (_i32, [_vp, _u32, _u32, _VPP]),
    "pfx_ct_destroy": (None, [_vp]),
    "pfx_ct_info": (_i32, [_vp, _IP]),
    "pfx_ct_set_scale": (_i32, [_vp, ctypes.c_double]),
    "pfx_ct_import": (_i32, [_vp, _u64p, _u32, _u32, ctypes.c_double, _vp, _vp]),
    "pfx_ct_export": (_i32, [_vp, _vp, _u64p, _sz, _IP, _vp]),
    "pfx_ct_copy": (_i32, [_vp, _vp, _vp, _vp]),
    "pfx_add": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "pfx_sub": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "pfx_neg": (_i32, [_vp, _vp, _vp, _vp]),
    "pfx_add_plain": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "pfx_mul_plain": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "pfx_mul_int": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "pfx_mul": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "pfx_mul_acc": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "pfx_mul_plain_acc": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "pfx_mul_int_acc": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "pfx_relinearize": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "pfx_mul_relin": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "pfx_mul_relin_batch": (_i32, [_vp, _VPP, _VPP, _sz, _vp, _VPP, _vp]),
    "pfx_mul_relin_noalloc": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "pfx_noalloc_scratch_bytes": (_sz, []),
    "pfx_rescale": (_i32, [_vp, _vp, _vp, _vp]),
    "pfx_rescale_batch": (_i32, [_vp, _VPP, _sz, _VPP, _vp]),
    "pfx_relinearize_batch": (_i32, [_vp, _VPP, _sz, _vp, _VPP, _vp]),
    "pfx_drop_level": (_i32, [_vp, _vp, _u32, _vp, _vp]),
    "pfx_key_switch": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "pfx_apply_galois": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "pfx_apply_galois_batch": (_i32, [_vp, _VPP, _sz, _vp, _VPP, _vp]),
    "pfx_rotate_batch": (_i32, [_vp, _VPP, _vp, _sz, _VPP, _sz, _VPP, _vp]),
    "pfx_mul_monomial": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "pfx_mul_inv_n": (_i32, [_vp, _vp, _vp, _vp]),
    "pfx_repack": (_i32, [_vp, _VPP, _sz, _VPP, _sz, _VPP, _vp]),
    "pfx_apply_galois_hoisted": (_i32, [_vp, _vp, _VPP, _sz, _VPP, _vp]),
    "pfx_linear_transform": (_i32, [_vp, _vp, _VPP, _vp, _sz, _u32, _VPP, _sz, _vp, _vp]),
    "pfx_pfe_repack": (_i32, [_vp, _VPP, _sz, _vp, _sz, _VPP, _sz, _VPP, _vp]),
    "pfx_ring_merge": (_i32, [_vp, _vp, _VPP, _sz, _vp, _vp, _vp]),
    "pfx_mod_raise": (_i32, [_vp, _vp, _u32, _vp, _vp]),
    "pfx_subring_trace": (_i32, [_vp, _vp, _u32, _VPP, _sz, _vp, _vp]),
    "pfx_swk_create_from": (_i32, [_vp, _vp, _vp, _u64p, _i64p, _VPP]),
    "pfx_rotate": (_i32, [_vp, _vp, _i32, _VPP, _sz, _vp, _vp]),
    "pfx_conjugate": (_i32, [_vp, _vp, _VPP, _sz, _vp, _vp]),
    "pfx_rotate_sum": (_i32, [_vp, _vp, _u32, _VPP, _sz, _vp, _vp]),
    "pfx_ntt": (_i32, [_vp, _vp, _u32, _u32, _sz, ctypes.c_int, _vp]),
    "pfx_add_const": (_i32, [_vp, _vp, ctypes.c_double, _vp, _vp]),
    "pfx_mul_const": (_i32, [_vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp]),
    "pfx_run_circuit": (_i32, [_vp, ctypes.POINTER(pfx_op), _sz, _VPP, _sz, _sz, _VPP, _sz, _vp, _VPP, _sz,
                               ctypes.c_int, _vp]),
    "pfx_batch_mul_relin_rescale": (_i32, [_VPP, _VPP, _VPP, _VPP, _VPP, _sz, ctypes.c_int, _vp]),
    "pfx_ctx_set_allocator": (_i32, [_vp, _vp, _vp, _vp, _sz]),
    "pfx_ctx_mem": (_i32, [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "pfx_tuning_set": (_i32, [ctypes.POINTER(pfx_pass_tuning)]),
    "pfx_tuning_get": (_i32, [_u32, ctypes.POINTER(pfx_pass_tuning)]),
    "pfx_tuning_reset": (_i32, []),
    "pfx_tuning_load": (_i32, [ctypes.c_char_p]),
    "pfx_graph_cache_stats": (_i32, [ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_uint64)]),
    "pfx_server_create": (_i32, [_vp, _sz, _u32, _u32, _vp, _VPP, _sz, _VPP]),
    "pfx_server_submit": (_i32, [_vp, ctypes.POINTER(pfx_request), ctypes.POINTER(ctypes.c_uint64)]),
    "pfx_server_poll": (_i32, [_vp, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(pfx_request_info)]),
    "pfx_server_stats_get": (_i32, [_vp, ctypes.POINTER(pfx_server_stats)]),
    "pfx_server_destroy": (None, [_vp]),
    "pfx_dev_alloc": (_i32, [_vp, _sz, _VPP]),
    "pfx_dev_free": (_i32, [_vp, _vp]),
    "pfx_memcpy_htod": (_i32, [_vp, _vp, _vp, _sz, _vp]),
    "pfx_memcpy_dtoh": (_i32, [_vp, _vp, _vp, _sz, _vp]),
    "pfx_stream_create": (_i32, [_vp, _VPP]),
    "pfx_stream_destroy": (_i32, [_vp, _vp]),
    "pfx_event_create": (_i32, [_vp, _VPP]),
    "pfx_event_record": (_i32, [_vp, _vp, _vp]),
    "pfx_stream_wait_event": (_i32, [_vp, _vp, _vp]),
    "pfx_event_elapsed": (_i32, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_float)]),
    "pfx_event_destroy": (_i32, [_vp, _vp]),
    "pfx_profile_enable": (_i32, [_vp, ctypes.c_int]),
    "pfx_profile_get": (_i32, [_vp, ctypes.c_char_p, _u64p, _f64p, _f64p]),
    "pfx_profile_names": (_i32, [_vp, ctypes.c_char_p, _sz]),
    "pfx_profile_reset": (_i32, [_vp]),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols():
    return list(_SIGS)


def _check(st: int):
    if st != PFX_OK:
        raise PfxError(st, _lib.pfx_last_error().decode())


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(_u64p)


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_i64p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_f64p)


def _stream(s):
    return None if s is None else ctypes.c_void_p(int(s))


def _keys(keys):
    arr = (ctypes.c_void_p * max(1, len(keys)))(*[k for k in keys])
    return arr, len(keys)


def make_params(log_n, q_bits, p_bits, alpha, mod_log2=0) -> pfx_params:
    p = pfx_params()
    p.log_n, p.n_q, p.n_p, p.alpha, p.mod_log2 = log_n, len(q_bits), len(p_bits), alpha, mod_log2
    for i, b in enumerate(q_bits):
        p.q_bits[i] = b
    for i, b in enumerate(p_bits):
        p.p_bits[i] = b
    return p


# ---------------------------------------------------------------- host only
def pfx_status_str(st: int) -> str:
    return _lib.pfx_status_str(st).decode()


def pfx_params_primes(prm: pfx_params):
    q = np.zeros(prm.n_q, np.uint64)
    p = np.zeros(prm.n_p, np.uint64)
    psi = np.zeros(prm.n_q + prm.n_p, np.uint64)
    _check(_lib.pfx_params_primes(ctypes.byref(prm), _u64(q)[1], _u64(p)[1], _u64(psi)[1]))
    return q, p, psi


def pfx_encode_words(prm: pfx_params, re, im, n_limbs: int, scale: float) -> np.ndarray:
    re_a, re_p = _f64(re)
    im_a, im_p = (None, None) if im is None else _f64(im)
    out = np.zeros((n_limbs, 1 << prm.log_n), np.uint64)
    _check(_lib.pfx_encode_words(ctypes.byref(prm), re_p, im_p, len(re_a), n_limbs, scale, _u64(out)[1]))
    return out


def pfx_decode_words(prm: pfx_params, words, scale: float, n_slots: int) -> np.ndarray:
    w, wp = _u64(words)
    re = np.zeros(n_slots)
    im = np.zeros(n_slots)
    _check(_lib.pfx_decode_words(ctypes.byref(prm), wp, w.shape[0], scale, _f64(re)[1], _f64(im)[1], n_slots))
    return re + 1j * im


# ---------------------------------------------------------------- context and keys
def pfx_ctx_create(prm: pfx_params, device: int = 0):
    h = ctypes.c_void_p()
    _check(_lib.pfx_ctx_create(ctypes.byref(prm), device, ctypes.byref(h)))
    return h.value


def pfx_ctx_destroy(ctx):
    _lib.pfx_ctx_destroy(ctx)


def pfx_ctx_moduli(ctx, n_q: int, n_p: int):
    q = np.zeros(n_q, np.uint64)
    p = np.zeros(n_p, np.uint64)
    psi = np.zeros(n_q + n_p, np.uint64)
    _check(_lib.pfx_ctx_moduli(ctx, _u64(q)[1], _u64(p)[1], _u64(psi)[1]))
    return q, p, psi


def pfx_sync(ctx, stream=None):
    _check(_lib.pfx_sync(ctx, _stream(stream)))


def pfx_sk_create(ctx, s):
    s = np.ascontiguousarray(s, dtype=np.int8)
    h = ctypes.c_void_p()
    _check(_lib.pfx_sk_create(ctx, s.ctypes.data_as(_i8p), ctypes.byref(h)))
    return h.value


def pfx_sk_destroy(sk):
    _lib.pfx_sk_destroy(sk)


def pfx_swk_create(ctx, sk, galois: int, a, e):
    a_, ap = _u64(a)
    e_, ep = _i64(e)
    h = ctypes.c_void_p()
    _check(_lib.pfx_swk_create(ctx, sk, galois, ap, ep, ctypes.byref(h)))
    return h.value


def pfx_swk_create_from(ctx, sk, s_from, a, e):
    s8 = np.ascontiguousarray(np.asarray(s_from, dtype=np.int8))
    a_, ap = _u64(a)
    e_, ep = _i64(e)
    h = ctypes.c_void_p()
    _check(_lib.pfx_swk_create_from(ctx, sk, s8.ctypes.data_as(_vp), ap, ep, ctypes.byref(h)))
    return h.value


def pfx_swk_export(ctx, k, beta: int, n_primes: int, n: int) -> np.ndarray:
    out = np.zeros((beta, 2, n_primes, n), np.uint64)
    _check(_lib.pfx_swk_export(ctx, k, _u64(out)[1], out.size))
    return out


def pfx_swk_galois(k) -> int:
    return _lib.pfx_swk_galois(k)


def _seed(seed: bytes):
    seed = bytes(seed)
    if len(seed) != 32:
        raise ValueError("seeds are 32 bytes")
    return ctypes.create_string_buffer(seed, 32)


def pfx_swk_import(ctx, galois: int, words):
    w = np.ascontiguousarray(words, dtype=np.uint64)
    h = ctypes.c_void_p()
    _check(_lib.pfx_swk_import(ctx, galois, _u64(w)[1], w.size, ctypes.byref(h)))
    return h.value


def pfx_sk_export(sk, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.int8)
    _check(_lib.pfx_sk_export(sk, out.ctypes.data, n))
    return out


def pfx_keygen_secret(ctx, seed: bytes, h: int):
    out = ctypes.c_void_p()
    _check(_lib.pfx_keygen_secret(ctx, _seed(seed), h, ctypes.byref(out)))
    return out.value


def pfx_keygen_relin(ctx, sk, seed: bytes):
    out = ctypes.c_void_p()
    _check(_lib.pfx_keygen_relin(ctx, sk, _seed(seed), ctypes.byref(out)))
    return out.value


def pfx_keygen_galois(ctx, sk, steps, conj: bool, seed: bytes):
    st = np.ascontiguousarray(steps, dtype=np.int32)
    n = st.size + (1 if conj else 0)
    outs = (ctypes.c_void_p * max(1, n))()
    _check(_lib.pfx_keygen_galois(ctx, sk, st.ctypes.data if st.size else None, st.size, int(bool(conj)),
                                  _seed(seed), outs))
    return [outs[i] for i in range(n)]


def pfx_encrypt_seeded(ctx, sk, pt, seed: bytes, out, stream=None):
    _check(_lib.pfx_encrypt_seeded(ctx, sk, pt, _seed(seed), out, _stream(stream)))


def pfx_shake256(msg: bytes, outlen: int) -> bytes:
    buf = ctypes.create_string_buffer(bytes(msg), max(1, len(msg)))
    out = ctypes.create_string_buffer(max(1, outlen))
    _check(_lib.pfx_shake256(buf, len(msg), out, outlen))
    return out.raw[:outlen]


def pfx_sample_uniform(seed: bytes, tag: int, index: int, limb: int, q: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    _check(_lib.pfx_sample_uniform(_seed(seed), tag, index, limb, q, n, _u64(out)[1]))
    return out


def pfx_sample_secret(seed: bytes, n: int, h: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.int8)
    _check(_lib.pfx_sample_secret(_seed(seed), n, h, out.ctypes.data))
    return out


def pfx_sample_gaussian(seed: bytes, tag: int, index: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.int64)
    _check(_lib.pfx_sample_gaussian(_seed(seed), tag, index, n, _i64(out)[1]))
    return out


def pfx_swk_destroy(k):
    _lib.pfx_swk_destroy(k)


# ---------------------------------------------------------------- plaintexts, encryption
def pfx_encode(ctx, re, im, n_limbs: int, scale: float):
    re_a, re_p = _f64(re)
    im_a, im_p = (None, None) if im is None else _f64(im)
    h = ctypes.c_void_p()
    _check(_lib.pfx_encode(ctx, re_p, im_p, len(re_a), n_limbs, scale, ctypes.byref(h)))
    return h.value


def pfx_decode(ctx, pt, n_slots: int) -> np.ndarray:
    re = np.zeros(n_slots)
    im = np.zeros(n_slots)
    _check(_lib.pfx_decode(ctx, pt, _f64(re)[1], _f64(im)[1], n_slots))
    return re + 1j * im


def pfx_pt_import(ctx, words, scale: float):
    w, wp = _u64(words)
    h = ctypes.c_void_p()
    _check(_lib.pfx_pt_import(ctx, wp, w.shape[0], scale, ctypes.byref(h)))
    return h.value


def pfx_encrypt(ctx, sk, pt, a, e, out, stream=None):
    a_, ap = _u64(a)
    e_, ep = _i64(e)
    _check(_lib.pfx_encrypt(ctx, sk, pt, ap, ep, out, _stream(stream)))


def pfx_decrypt(ctx, sk, ct, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.pfx_decrypt(ctx, sk, ct, ctypes.byref(h), _stream(stream)))
    return h.value


# ---------------------------------------------------------------- ciphertexts
def pfx_ct_create(ctx, cap_limbs: int, cap_degree: int = 1):
    h = ctypes.c_void_p()
    _check(_lib.pfx_ct_create(ctx, cap_limbs, cap_degree, ctypes.byref(h)))
    return h.value


def pfx_ct_destroy(ct):
    _lib.pfx_ct_destroy(ct)


def pfx_ct_info(ct) -> pfx_info:
    info = pfx_info()
    _check(_lib.pfx_ct_info(ct, ctypes.byref(info)))
    return info


def pfx_ct_set_scale(ct, scale: float):
    _check(_lib.pfx_ct_set_scale(ct, scale))


def pfx_ct_import(ctx, words, scale: float, out, stream=None):
    w, wp = _u64(words)
    assert w.ndim == 3
    _check(_lib.pfx_ct_import(ctx, wp, w.shape[1], w.shape[0] - 1, scale, out, _stream(stream)))


def pfx_ct_export(ctx, ct, n: int, stream=None) -> np.ndarray:
    info = pfx_ct_info(ct)
    out = np.zeros((info.degree + 1, info.n_limbs, n), np.uint64)
    _check(_lib.pfx_ct_export(ctx, ct, _u64(out)[1], out.size, None, _stream(stream)))
    return out


def pfx_ct_copy(ctx, src, dst, stream=None):
    _check(_lib.pfx_ct_copy(ctx, src, dst, _stream(stream)))


# ---------------------------------------------------------------- evaluation
def pfx_add(ctx, a, b, out, stream=None):
    _check(_lib.pfx_add(ctx, a, b, out, _stream(stream)))


def pfx_sub(ctx, a, b, out, stream=None):
    _check(_lib.pfx_sub(ctx, a, b, out, _stream(stream)))


def pfx_neg(ctx, a, out, stream=None):
    _check(_lib.pfx_neg(ctx, a, out, _stream(stream)))


def pfx_add_plain(ctx, a, m, out, stream=None):
    _check(_lib.pfx_add_plain(ctx, a, m, out, _stream(stream)))


def pfx_mul_plain(ctx, a, m, out, stream=None):
    _check(_lib.pfx_mul_plain(ctx, a, m, out, _stream(stream)))


def pfx_mul_int(ctx, a, k: int, out, stream=None):
    _check(_lib.pfx_mul_int(ctx, a, k, out, _stream(stream)))


def pfx_mul(ctx, a, b, out, stream=None):
    _check(_lib.pfx_mul(ctx, a, b, out, _stream(stream)))


def pfx_mul_acc(ctx, a, b, acc, stream=None):
    _check(_lib.pfx_mul_acc(ctx, a, b, acc, _stream(stream)))


def pfx_mul_plain_acc(ctx, a, m, acc, stream=None):
    _check(_lib.pfx_mul_plain_acc(ctx, a, m, acc, _stream(stream)))


def pfx_mul_int_acc(ctx, a, k: int, acc, stream=None):
    _check(_lib.pfx_mul_int_acc(ctx, a, k, acc, _stream(stream)))


def pfx_relinearize(ctx, a, rlk, out, stream=None):
    _check(_lib.pfx_relinearize(ctx, a, rlk, out, _stream(stream)))


def pfx_mul_relin(ctx, a, b, rlk, out, stream=None):
    _check(_lib.pfx_mul_relin(ctx, a, b, rlk, out, _stream(stream)))


def pfx_mul_relin_noalloc(ctx, a, b, rlk, out, stream=None):
    _check(_lib.pfx_mul_relin_noalloc(ctx, a, b, rlk, out, _stream(stream)))


def pfx_noalloc_scratch_bytes() -> int:
    return int(_lib.pfx_noalloc_scratch_bytes())


def pfx_mul_relin_batch(ctx, a, b, rlk, outs, stream=None):
    n = len(a)
    assert len(b) == n and len(outs) == n
    arr = lambda xs: (ctypes.c_void_p * max(1, n))(*xs)
    _check(_lib.pfx_mul_relin_batch(ctx, arr(a), arr(b), n, rlk, arr(outs), _stream(stream)))


def pfx_rescale(ctx, a, out, stream=None):
    _check(_lib.pfx_rescale(ctx, a, out, _stream(stream)))


def pfx_relinearize_batch(ctx, a, rlk, outs, stream=None):
    n = len(a)
    assert len(outs) == n
    arr = lambda xs: (ctypes.c_void_p * max(1, n))(*xs)
    _check(_lib.pfx_relinearize_batch(ctx, arr(a), n, rlk, arr(outs), _stream(stream)))


def pfx_rescale_batch(ctx, a, outs, stream=None):
    n = len(a)
    assert len(outs) == n
    arr = lambda xs: (ctypes.c_void_p * max(1, n))(*xs)
    _check(_lib.pfx_rescale_batch(ctx, arr(a), n, arr(outs), _stream(stream)))


def pfx_drop_level(ctx, a, n_limbs: int, out, stream=None):
    _check(_lib.pfx_drop_level(ctx, a, n_limbs, out, _stream(stream)))


def pfx_key_switch(ctx, d, k, out, stream=None):
    _check(_lib.pfx_key_switch(ctx, d, k, out, _stream(stream)))


def pfx_apply_galois(ctx, a, gk, out, stream=None):
    _check(_lib.pfx_apply_galois(ctx, a, gk, out, _stream(stream)))


def pfx_apply_galois_batch(ctx, a, gk, outs, stream=None):
    n = len(a)
    assert len(outs) == n
    arr = lambda xs: (ctypes.c_void_p * max(1, n))(*xs)
    _check(_lib.pfx_apply_galois_batch(ctx, arr(a), n, gk, arr(outs), _stream(stream)))


def pfx_rotate_batch(ctx, a, steps, gks, outs, stream=None):
    """outs[i] = rotate(a[i], steps[i]) with the key for each step among gks."""
    n = len(a)
    assert len(steps) == n and len(outs) == n
    arr = lambda xs: (ctypes.c_void_p * max(1, len(xs)))(*xs)
    st = np.ascontiguousarray(steps, dtype=np.int32)
    _check(_lib.pfx_rotate_batch(ctx, arr(a), st.ctypes.data if n else None, n, arr(gks), len(gks), arr(outs),
                                 _stream(stream)))


def pfx_apply_galois_hoisted(ctx, a, gks, outs, stream=None):
    G = (ctypes.c_void_p * max(1, len(gks)))(*gks)
    O = (ctypes.c_void_p * max(1, len(outs)))(*outs)
    assert len(gks) == len(outs)
    _check(_lib.pfx_apply_galois_hoisted(ctx, a, G, len(gks), O, _stream(stream)))


def pfx_linear_transform(ctx, a, diags, steps, n1: int, keys, out, stream=None):
    D = (ctypes.c_void_p * max(1, len(diags)))(*diags)
    st = np.ascontiguousarray(np.asarray(steps, dtype=np.int32))
    assert len(st) == len(diags)
    K, nk = _keys(keys)
    _check(_lib.pfx_linear_transform(ctx, a, D, st.ctypes.data_as(_vp), len(diags), n1, K, nk, out,
                                     _stream(stream)))


def pfx_mul_monomial(ctx, a, k: int, out, stream=None):
    _check(_lib.pfx_mul_monomial(ctx, a, k, out, _stream(stream)))


def pfx_mul_inv_n(ctx, a, out, stream=None):
    _check(_lib.pfx_mul_inv_n(ctx, a, out, _stream(stream)))


def pfx_repack(ctx, cts, gks, outs, stream=None):
    n = len(cts)
    arr = (ctypes.c_void_p * max(1, n))(*cts)
    O = (ctypes.c_void_p * max(1, len(outs)))(*outs)
    K, nk = _keys(gks)
    _check(_lib.pfx_repack(ctx, arr, n, K, nk, O, _stream(stream)))


def pfx_pfe_repack(ctx, tables, d_exps: int, n: int, gks, outs, stream=None):
    """d_exps: device pointer to n * len(tables) int64 exponents (row-major by record)."""
    T = (ctypes.c_void_p * max(1, len(tables)))(*tables)
    O = (ctypes.c_void_p * max(1, len(outs)))(*outs)
    K, nk = _keys(gks)
    _check(_lib.pfx_pfe_repack(ctx, T, len(tables), d_exps, n, K, nk, O, _stream(stream)))


def pfx_mod_raise(ctx, a, n_limbs: int, out, stream=None):
    _check(_lib.pfx_mod_raise(ctx, a, n_limbs, out, _stream(stream)))


def pfx_subring_trace(ctx, a, log_r: int, keys, out, stream=None):
    K, nk = _keys(keys)
    _check(_lib.pfx_subring_trace(ctx, a, log_r, K, nk, out, _stream(stream)))


def pfx_ring_merge(big, small, cts, swk, out, stream=None):
    arr = (ctypes.c_void_p * max(1, len(cts)))(*cts)
    _check(_lib.pfx_ring_merge(big, small, arr, len(cts), swk, out, _stream(stream)))


def pfx_rotate(ctx, a, step: int, keys, out, stream=None):
    arr, n = _keys(keys)
    _check(_lib.pfx_rotate(ctx, a, step, arr, n, out, _stream(stream)))


def pfx_conjugate(ctx, a, keys, out, stream=None):
    arr, n = _keys(keys)
    _check(_lib.pfx_conjugate(ctx, a, arr, n, out, _stream(stream)))


def pfx_rotate_sum(ctx, a, log_steps: int, keys, out, stream=None):
    arr, n = _keys(keys)
    _check(_lib.pfx_rotate_sum(ctx, a, log_steps, arr, n, out, _stream(stream)))


def pfx_ntt(ctx, d_words_ptr: int, first_prime: int, n_limbs: int, batch: int, inverse: bool, stream=None):
    _check(_lib.pfx_ntt(ctx, ctypes.c_void_p(d_words_ptr), first_prime, n_limbs, batch, int(inverse),
                        _stream(stream)))


def pfx_add_const(ctx, a, value: float, out, stream=None):
    _check(_lib.pfx_add_const(ctx, a, value, out, _stream(stream)))


def pfx_mul_const(ctx, a, value: float, cscale: float, out, stream=None):
    _check(_lib.pfx_mul_const(ctx, a, value, cscale, out, _stream(stream)))


RUN_EAGER, RUN_GRAPH, RUN_LANES = 0, 1, 2


def pfx_run_circuit(ctx, ops, regs, n_inputs: int, pts, rlk, gks, mode: int = RUN_EAGER, stream=None):
    """ops: a sequence of (code, dst, a, b, k, value); mode: RUN_* flags (a bool
    selects RUN_GRAPH or RUN_EAGER)."""
    arr = (pfx_op * max(1, len(ops)))(*[pfx_op(*o) for o in ops])
    R = (ctypes.c_void_p * max(1, len(regs)))(*regs)
    Pt = (ctypes.c_void_p * max(1, len(pts)))(*pts)
    G = (ctypes.c_void_p * max(1, len(gks)))(*gks)
    _check(_lib.pfx_run_circuit(ctx, arr, len(ops), R, len(regs), n_inputs, Pt, len(pts), rlk, G, len(gks),
                                int(mode), _stream(stream)))


def pfx_batch_mul_relin_rescale(ctxs, a, b, rlks, outs, mode: int, stream=None):
    n = len(a)
    arr = lambda xs: (ctypes.c_void_p * max(1, n))(*xs)
    _check(_lib.pfx_batch_mul_relin_rescale(arr(ctxs), arr(a), arr(b), arr(rlks), arr(outs), n, mode,
                                            _stream(stream)))


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


_CALLBACKS = []   # every allocator thunk handed to the library: memory made through one is freed through it


def pfx_ctx_set_allocator(ctx, alloc=None, free=None, budget: int = 0):
    """alloc(bytes, stream) -> device pointer or 0, free(ptr, stream): Python
    callables (both or neither; their C thunks are kept for the life of the
    process, since memory is freed through the thunk that made it); budget:
    bytes the context may hold (0 = no cap)."""
    fa = ALLOC_FN(lambda n, st, u: alloc(n, st) or None) if alloc else None
    ff = FREE_FN(lambda p, st, u: free(p, st)) if free else None
    _CALLBACKS.append((fa, ff))
    _check(_lib.pfx_ctx_set_allocator(ctx, ctypes.cast(fa, ctypes.c_void_p) if fa else None,
                                      ctypes.cast(ff, ctypes.c_void_p) if ff else None, None, int(budget)))
    return (fa, ff)


def pfx_ctx_mem(ctx):
    """(bytes held now, most bytes held so far) of the context's device memory."""
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.pfx_ctx_mem(ctx, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


TUNING_FIELDS = ("row_wg256", "col_wg256", "widen_wg", "min_col", "min_col_special", "rs_widen_wg", "ks_fuse",
                 "ks_batch", "ks_modup_batch")


def pfx_tuning_set(log_n: int, **fields):
    """Pass geometry for ring degree 2^log_n; fields not given keep their value."""
    t = pfx_tuning_get(log_n)
    for k, v in fields.items():
        setattr(t, k, int(v))
    _check(_lib.pfx_tuning_set(ctypes.byref(t)))


def pfx_tuning_get(log_n: int) -> pfx_pass_tuning:
    t = pfx_pass_tuning()
    _check(_lib.pfx_tuning_get(log_n, ctypes.byref(t)))
    return t


def pfx_tuning_reset():
    _check(_lib.pfx_tuning_reset())


def pfx_tuning_load(path: str):
    _check(_lib.pfx_tuning_load(path.encode()))


def pfx_graph_cache_stats():
    """(entries held, captures made) of the process-wide graph cache."""
    e, c = ctypes.c_size_t(), ctypes.c_uint64()
    _check(_lib.pfx_graph_cache_stats(ctypes.byref(e), ctypes.byref(c)))
    return e.value, c.value


# ---------------------------------------------------------------- served form
def pfx_server_create(ctx, hbm_budget: int, slots: int, rlk, gks, max_batch: int = 1):
    G = (ctypes.c_void_p * max(1, len(gks)))(*gks)
    h = ctypes.c_void_p()
    _check(_lib.pfx_server_create(ctx, hbm_budget, slots, max_batch, rlk, G, len(gks), ctypes.byref(h)))
    return h.value


def pfx_server_submit(srv, ops, n_regs: int, inputs, pts, out_reg: int, out, reg_degree=None) -> int:
    """ops: a sequence of (code, dst, a, b, k, value); inputs are registers 0..len(inputs)-1;
    reg_degree: capacity degree (1 or 2) per register, None for all 1."""
    arr = (pfx_op * max(1, len(ops)))(*[pfx_op(*o) for o in ops])
    I = (ctypes.c_void_p * max(1, len(inputs)))(*inputs)
    Pt = (ctypes.c_void_p * max(1, len(pts)))(*pts)
    D = None
    if reg_degree is not None:
        assert len(reg_degree) == n_regs
        D = (ctypes.c_uint8 * max(1, n_regs))(*reg_degree)
    rq = pfx_request(arr, len(ops), n_regs, len(inputs), I, Pt, len(pts), out_reg, out,
                     ctypes.cast(D, ctypes.POINTER(ctypes.c_uint8)) if D is not None else None)
    t = ctypes.c_uint64()
    _check(_lib.pfx_server_submit(srv, ctypes.byref(rq), ctypes.byref(t)))
    return t.value


def pfx_server_poll(srv, ticket: int, wait: bool = False):
    """The finished request's pfx_request_info, or None while it is queued or running."""
    info = pfx_request_info()
    st = _lib.pfx_server_poll(srv, ticket, int(wait), ctypes.byref(info))
    if st == PFX_EBUSY:
        return None
    _check(st)
    return info


def pfx_server_stats_get(srv) -> dict:
    st = pfx_server_stats()
    _check(_lib.pfx_server_stats_get(srv, ctypes.byref(st)))
    return {n: getattr(st, n) for n, _ in pfx_server_stats._fields_}


def pfx_server_destroy(srv):
    _lib.pfx_server_destroy(srv)


# ---------------------------------------------------------------- plumbing
def pfx_dev_alloc(ctx, nbytes: int) -> int:
    h = ctypes.c_void_p()
    _check(_lib.pfx_dev_alloc(ctx, nbytes, ctypes.byref(h)))
    return h.value


def pfx_dev_free(ctx, ptr: int):
    _check(_lib.pfx_dev_free(ctx, ctypes.c_void_p(ptr)))


def pfx_memcpy_htod(ctx, dst: int, arr: np.ndarray, stream=None):
    arr = np.ascontiguousarray(arr)
    _check(_lib.pfx_memcpy_htod(ctx, ctypes.c_void_p(dst), arr.ctypes.data_as(_vp), arr.nbytes, _stream(stream)))


def pfx_memcpy_dtoh(ctx, arr: np.ndarray, src: int, stream=None):
    assert arr.flags["C_CONTIGUOUS"]
    _check(_lib.pfx_memcpy_dtoh(ctx, arr.ctypes.data_as(_vp), ctypes.c_void_p(src), arr.nbytes, _stream(stream)))


def pfx_stream_create(ctx) -> int:
    h = ctypes.c_void_p()
    _check(_lib.pfx_stream_create(ctx, ctypes.byref(h)))
    return h.value


def pfx_stream_destroy(ctx, stream: int):
    _check(_lib.pfx_stream_destroy(ctx, ctypes.c_void_p(stream)))


def pfx_event_create(ctx) -> int:
    h = ctypes.c_void_p()
    _check(_lib.pfx_event_create(ctx, ctypes.byref(h)))
    return h.value


def pfx_event_record(ctx, event: int, stream=None):
    _check(_lib.pfx_event_record(ctx, ctypes.c_void_p(event), _stream(stream)))


def pfx_stream_wait_event(ctx, stream, event: int):
    _check(_lib.pfx_stream_wait_event(ctx, _stream(stream), ctypes.c_void_p(event)))


def pfx_event_elapsed(ctx, start: int, end: int) -> float:
    ms = ctypes.c_float()
    _check(_lib.pfx_event_elapsed(ctx, ctypes.c_void_p(start), ctypes.c_void_p(end), ctypes.byref(ms)))
    return ms.value


def pfx_event_destroy(ctx, event: int):
    _check(_lib.pfx_event_destroy(ctx, ctypes.c_void_p(event)))


# ---------------------------------------------------------------- profiling
def pfx_profile_enable(ctx, on: bool = True):
    _check(_lib.pfx_profile_enable(ctx, int(on)))


def pfx_profile_get(ctx, kernel: str):
    """(launches, total device ms, total algorithmic bytes) of one kernel name."""
    n = ctypes.c_uint64()
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(_lib.pfx_profile_get(ctx, kernel.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return n.value, ms.value, by.value


def pfx_profile_names(ctx):
    buf = ctypes.create_string_buffer(8192)
    _check(_lib.pfx_profile_names(ctx, buf, len(buf)))
    return [s for s in buf.value.decode().split("\n") if s]


def pfx_profile_reset(ctx):
    _check(_lib.pfx_profile_reset(ctx))
