"""ctypes binding of libhypercurves.so (include/hypercurves.h), same names.

Argument marshalling only: every step of the search runs in the library's HIP
kernels.  If the library is missing this module raises -- there is no CPU
fallback.
"""
import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhypercurves.so")

HC_OK, HC_ERR_INVALID, HC_ERR_SIZE, HC_ERR_HIP, HC_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
HC_K_MAX = 256
HC_PATH_AUTO, HC_PATH_GATHER, HC_PATH_BAND = 0, 1, 2
HC_NOALLOC_SCRATCH_BYTES = 4 << 20
HC_BAND_K_MAX = 128


class HcError(RuntimeError):
    def __init__(self, name, status):
        self.status = status
        super().__init__(f"{name} failed: {status_str(status)} ({status})")


class hc_uneven_cfg(ct.Structure):
    _fields_ = [("chunk_slots", ct.c_uint32), ("max_split", ct.c_uint32),
                ("blocks_per_cu", ct.c_uint32)]


class hc_params(ct.Structure):
    _fields_ = [("dim", ct.c_uint32), ("curves", ct.c_uint32),
                ("dims_per_curve", ct.c_uint32), ("bits", ct.c_uint32),
                ("perm", ct.POINTER(ct.c_uint16)), ("curve", ct.c_uint32)]


_vp = ct.c_void_p
_u32 = ct.c_uint32
_u64 = ct.c_uint64
_sz = ct.c_size_t
_pp = ct.POINTER(hc_params)

# name -> argtypes (every function returns hc_status, an int)
SIGNATURES = {
    "hc_index_bytes": [_pp, _u64, ct.POINTER(_sz), ct.POINTER(_sz)],
    "hc_build_index": [_pp, _vp, _u64, _vp, _sz, _vp, _sz, _vp, ct.POINTER(_vp)],
    "hc_index_attach": [_pp, _vp, _u64, _vp, _sz, ct.POINTER(_vp)],
    "hc_insert_bytes": [_vp, _u64, ct.POINTER(_sz), ct.POINTER(_sz)],
    "hc_host_index_bytes": [_vp, ct.POINTER(_sz)],
    "hc_rowstore_bytes": [_vp, ct.POINTER(_sz)],
    "hc_rowstore_build": [_vp, _vp, _sz, _vp],
    "hc_rowstore_detach": [_vp],
    "hc_host_index_copy": [_vp, _vp, _sz, _vp],
    "hc_host_search": [_vp, _vp, _vp, _vp, _u32, _u32, _vp, _u32, _vp, _u32, _vp, _vp],
    "hc_insert_rows": [_vp, _vp, _u64, _vp, _sz, _vp, _sz, _vp, ct.POINTER(_vp)],
    "hc_index_destroy": [_vp],
    "hc_index_curve": [_vp, _u32, ct.POINTER(_vp), ct.POINTER(_vp)],
    "hc_index_info": [_vp, ct.POINTER(_u64), ct.POINTER(_u32)],
    "hc_search_scratch_bytes": [_vp, _u32, ct.POINTER(_sz)],
    "hc_search_scratch_bytes_k": [_vp, _u32, _u32, ct.POINTER(_sz)],
    "hc_search_batch": [_vp, _vp, _u32, _u32, _u32, _vp, _vp, _vp, _vp, _sz, _vp],
    "hc_search_batch_noalloc": [_vp, _vp, _u32, _u32, _u32, _vp, _vp, _vp, _vp],
    "hc_encode_queries": [_vp, _vp, _u32, _vp, _sz, _vp],
    "hc_search_encoded": [_vp, _vp, _u32, _u32, _u32, _vp, _vp, _vp, _vp, _sz, _vp],
    "hc_search_choose_path": [_vp, _u32, _u32, _u32, _sz, ct.POINTER(_u32)],
    "hc_search_encoded_ex": [_vp, _vp, _u32, _u32, _u32, _vp, _vp, _vp, _vp, _sz, _u32, _vp],
    "hc_index_set_kernel_events": [_vp, _vp, _vp],
    "hc_encode_keys": [_pp, _vp, _u64, _vp, _vp],
    "hc_positions": [_vp, _vp, _u32, _vp, _vp, _sz, _vp],
    "hc_candidates": [_vp, _vp, _u32, _u32, _vp, _vp, _vp, _u32, _vp, _sz, _vp],
    "hc_brute_force_scratch_bytes": [_u64, _u32, _u32, ct.POINTER(_sz)],
    "hc_brute_force": [_vp, _u64, _vp, _u32, _u32, _vp, _vp, _vp, _sz, _vp],
    "hc_index_ranks": [_vp, _vp, _vp],
    "hc_labels": [_vp, _vp, _vp, _u32, _u32, _vp, _vp, _vp, _sz, _vp],
    "hc_union_sizes": [_vp, _vp, _vp, _u32, _u32, _vp, _vp, _vp, _sz, _vp],
    "hc_features": [_vp, _vp, _u32, _u32, _vp, _vp, _vp, _sz, _vp],
    "hc_mlp_infer": [_vp, _vp, _vp, _u32, ct.c_float, _u32, _u32, _u32, _vp, _vp, _vp],
    "hc_mlp_train_scratch_bytes": [_u32, ct.POINTER(_sz)],
    "hc_mlp_forward": [_vp, _vp, _vp, _vp, _u32, _vp, _vp],
    "hc_mlp_backward": [_vp, _vp, _vp, _vp, _vp, _u32, _vp, _vp, _vp, _sz, _vp],
    "hc_adam_step": [_vp, _vp, _vp, _vp, _u32, _u32, ct.c_float, ct.c_float, ct.c_float,
                     ct.c_float, _vp, _vp],
    "hc_to_bf16": [_vp, _u32, _vp, _vp],
    "hc_mlp_targets": [_vp, _u32, _u32, _u32, _vp, _vp],
    "hc_feature_norm": [_vp, _u32, _vp, _vp],
    "hc_uneven_scratch_bytes": [_vp, _u32, _u32, ct.POINTER(hc_uneven_cfg), ct.POINTER(_sz)],
    "hc_read_probe": [_vp, _sz, _vp, _u32, _vp],
    "hc_search_uneven": [_vp, _vp, _u32, _u32, _vp, _u32, _vp, _u32, _vp, _vp, _vp, _sz,
                         ct.POINTER(hc_uneven_cfg), _vp],
}

_LIB = None


def load():
    """The loaded library; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "(the search has no CPU fallback)")
        L = ct.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ct.c_int
        L.hc_status_str.argtypes = [ct.c_int]
        L.hc_status_str.restype = ct.c_char_p
        _LIB = L
    return _LIB


def status_str(status):
    return load().hc_status_str(status).decode()


def call(name, *args):
    """Calls an hc_ entry point and raises HcError on a non-zero status."""
    rc = getattr(load(), name)(*args)
    if rc != HC_OK:
        raise HcError(name, rc)
    return rc


CURVES = {"hilbert": 0, "zorder": 1}     # HC_CURVE_HILBERT, HC_CURVE_ZORDER


def make_params(dim=128, curves=8, dims_per_curve=16, bits=8, perm=None, curve="hilbert"):
    """hc_params plus the ctypes array that keeps `perm` alive."""
    p = hc_params(dim, curves, dims_per_curve, bits, None, CURVES[curve])
    keep = None
    if perm is not None:
        keep = (ct.c_uint16 * len(perm))(*[int(x) for x in perm])
        p.perm = ct.cast(keep, ct.POINTER(ct.c_uint16))
    return p, keep
