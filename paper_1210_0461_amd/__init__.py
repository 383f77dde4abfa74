"""MI355X column-row parallel (CRoP) library: Python binding.

A thin ctypes binding over the C ABI in ``include/crop.h``: every function
below has the name of the C function it calls and only marshals arguments
(tensor or array -> pointer, status -> exception).  All computation runs in
the HIP kernels of ``libcrop.so``; there is no Python or CPU fallback, and
importing this package fails loudly when the library has not been built
(``python -m paper_1210_0461_amd.build`` or ``__graft_entry__.build()``).

PyTorch is used only as a holder of device memory and streams.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrop.so")

CROP_MEM_HOST = 0
CROP_MEM_DEVICE = 1
CROP_OWN_COPY = 0
CROP_OWN_BORROW = 1

STATUS = {
    0: "CROP_OK", -1: "CROP_E_ARG", -2: "CROP_E_STATE", -3: "CROP_E_INPUT",
    -4: "CROP_E_CAPACITY", -5: "CROP_E_NOMEM", -6: "CROP_E_HIP", -7: "CROP_E_UNSUPPORTED",
}


class CropError(RuntimeError):
    def __init__(self, status: int, detail: str, index: int = -1):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status
        self.detail = detail
        self.index = index


class crop_stream_ref(ctypes.Structure):
    _fields_ = [("off", ctypes.c_void_p), ("T", ctypes.c_uint64), ("items", ctypes.c_void_p),
                ("nnz", ctypes.c_uint64), ("n_items", ctypes.c_uint32)]


class crop_train_set(ctypes.Structure):
    _fields_ = [("streams", ctypes.POINTER(crop_stream_ref)), ("n_streams", ctypes.c_uint32),
                ("where", ctypes.c_int)]


class crop_train_opts(ctypes.Structure):
    _fields_ = [("top_items", ctypes.c_uint32), ("epochs", ctypes.c_uint32),
                ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("shuffle_seed", ctypes.c_uint64), ("init", ctypes.c_void_p)]


class crop_tune(ctypes.Structure):
    _fields_ = [("bins_per_partition", ctypes.c_uint32), ("rows_per_chunk", ctypes.c_uint32),
                ("stage_keys", ctypes.c_uint32), ("route", ctypes.c_uint32),
                ("window", ctypes.c_uint32), ("region_terms", ctypes.c_uint32)]


# torch ships its own HIP runtime under the same soname (libamdhip64.so.7).
# Importing it first makes the dynamic loader bind libcrop.so to that one
# runtime instead of loading a second copy from /opt/rocm, so tensors, streams
# and this library share one HIP runtime in the process.
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is optional for the C ABI
    torch = None

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(the library has no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int
_pu64 = ctypes.POINTER(ctypes.c_uint64)

_SIGS = {
    "crop_abi_version": ([], _i32),
    "crop_status_string": ([_i32], ctypes.c_char_p),
    "crop_create": ([ctypes.POINTER(_vp), _i32], _i32),
    "crop_destroy": ([_vp], None),
    "crop_last_error_detail": ([_vp], ctypes.c_char_p),
    "crop_last_error_index": ([_vp], ctypes.c_int64),
    "crop_set_partitions": ([_vp, _u32], _i32),
    "crop_set_seed": ([_vp, _u64], _i32),
    "crop_set_summary": ([_vp, _u32, _u32], _i32),
    "crop_set_stream": ([_vp, _vp], _i32),
    "crop_use_own_stream": ([_vp], _i32),
    "crop_set_topk_rank": ([_vp, _i32], _i32),
    "crop_set_owned_partitions": ([_vp, _u32, _u32], _i32),
    "crop_set_tuning": ([_vp, ctypes.POINTER(crop_tune)], _i32),
    "crop_get_tuning": ([_vp, ctypes.POINTER(crop_tune)], _i32),
    "crop_load_transactions": ([_vp, _vp, _u64, _vp, _u64, _u32, _i32, _i32], _i32),
    "crop_load_outer": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _u64, _u64, _u64, _u32, _u32,
                         _i32, _i32], _i32),
    "crop_run_exact": ([_vp], _i32),
    "crop_result_sizes": ([_vp, _vp, _vp], _i32),
    "crop_read_partition": ([_vp, _u32, _vp, _vp, _vp, _vp, _u64, _pu64], _i32),
    "crop_read_all": ([_vp, _i32, _vp, _vp, _vp, _vp, _u64, _pu64, _vp], _i32),
    "crop_synchronize": ([_vp], _i32),
    "crop_last_run_ms": ([_vp, ctypes.POINTER(ctypes.c_float)], _i32),
    "crop_set_profiling": ([_vp, _i32], _i32),
    "crop_run_stages": ([_vp, _u32, ctypes.POINTER(_u32), _vp, _vp, _u32], _i32),
}

_SIGS.update({
    "crop_run_topk": ([_vp, _u32], _i32),
    "crop_run_topk_seeded": ([_vp, _u32, _vp, _vp, _u64, _u32], _i32),
    "crop_run_topk_amplified": ([_vp, _u32, _u32, _u32], _i32),
    "crop_autotune": ([_vp, _u32, _vp, _vp, _vp], _i32),
    "crop_read_topk_votes": ([_vp, _vp, _u64, _pu64], _i32),
    "crop_read_topk": ([_vp, _vp, _vp, _vp, _vp, _vp, _u64, _pu64], _i32),
    "crop_read_summary": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _u64, _pu64], _i32),
    "crop_run_countsketch": ([_vp, _u32, _u32], _i32),
    "crop_countsketch_estimate": ([_vp, _vp, _vp, _u64, _vp], _i32),
    "crop_read_countsketch": ([_vp, _u32, _vp, _u64], _i32),
    "crop_load_batch": ([_vp, _u32, _vp, _vp, _vp, _vp, _i32, _i32], _i32),
    "crop_batch_set_plan": ([_vp, _u32, _u32], _i32),
    "crop_batch_autotune": ([_vp, _u32, ctypes.POINTER(_u32), ctypes.POINTER(_u32),
                             ctypes.POINTER(ctypes.c_float)], _i32),
    "crop_batch_set_graph": ([_vp, _i32], _i32),
    "crop_run_exact_batched": ([_vp], _i32),
    "crop_batch_info": ([_vp, _u32, ctypes.POINTER(_u32), _pu64, _pu64, _pu64], _i32),
    "crop_batch_result_sizes": ([_vp, _u32, _vp, _vp], _i32),
    "crop_batch_read_stream": ([_vp, _u32, _i32, _vp, _vp, _vp, _u64, _pu64, _vp], _i32),
    "crop_item_features": ([_vp, _u32, _vp], _i32),
    "crop_item_features_noalloc": ([_vp, _u32, _vp], _i32),
    "crop_top_item_pairs": ([_vp, _u32, _u32, _vp, _vp, _u64, _pu64], _i32),
    "crop_lookup_exact": ([_vp, _vp, _vp, _u64, _vp], _i32),
    "crop_pair_inputs": ([_vp, _vp, _vp, _vp, _vp, _u64, _vp, _vp], _i32),
    "crop_mlp_create": ([_vp, _vp, ctypes.POINTER(_vp)], _i32),
    "crop_mlp_destroy": ([_vp], None),
    "crop_mlp_params": ([_vp, _vp, _vp], _i32),
    "crop_mlp_grad": ([_vp, _vp, _vp, _vp, _u32, _vp, _vp], _i32),
    "crop_mlp_train": ([_vp, _vp, _vp, _vp, _u64, _vp, _u64, _u32, ctypes.c_float], _i32),
    "crop_mlp_loss": ([_vp, _vp, _vp], _i32),
    "crop_mlp_score": ([_vp, _vp, _vp, _u64, _vp], _i32),
    "crop_select_seeds": ([_vp, _vp, _vp, _vp, _u64, _u32, _vp, _vp], _i32),
    "crop_hash_pairs": ([_vp, _vp, _vp, _u64, _vp, _vp], _i32),
    "crop_predictor_train": ([_vp, _vp, _vp, ctypes.POINTER(_vp)], _i32),
    "crop_predictor_score": ([_vp, _vp, _u32, _vp, _vp, _pu64], _i32),
    "crop_predictor_params": ([_vp, _vp, _vp, ctypes.POINTER(ctypes.c_float)], _i32),
    "crop_predictor_free": ([_vp], None),
})

# Entry points bound only when the loaded library exports them.
_OPTIONAL_SIGS: dict = {}

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res
for _name, (_args, _res) in _OPTIONAL_SIGS.items():
    if hasattr(_lib, _name):
        _f = getattr(_lib, _name)
        _f.argtypes = _args
        _f.restype = _res


def exported_symbols():
    """Names of the C functions this binding knows about."""
    return sorted(list(_SIGS) + [n for n in _OPTIONAL_SIGS if hasattr(_lib, n)])


# --------------------------------------------------------------------------
# marshalling helpers

def _ptr(a):
    """(pointer, where) of a torch tensor or numpy array (None -> NULL)."""
    if a is None:
        return None, CROP_MEM_HOST
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data, CROP_MEM_HOST
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), (CROP_MEM_DEVICE if a.is_cuda else CROP_MEM_HOST)
    if isinstance(a, int):
        return a, CROP_MEM_DEVICE
    raise TypeError(f"unsupported buffer type {type(a)}")


def _check(ctx, st):
    if st != 0:
        detail = _lib.crop_last_error_detail(ctx).decode() if ctx else ""
        idx = _lib.crop_last_error_index(ctx) if ctx else -1
        raise CropError(st, detail, idx)


# --------------------------------------------------------------------------
# the C ABI, one Python function per C function

def crop_abi_version() -> int:
    return _lib.crop_abi_version()


def crop_status_string(st: int) -> str:
    return _lib.crop_status_string(st).decode()


def crop_create(hip_device: int = 0):
    h = _vp()
    st = _lib.crop_create(ctypes.byref(h), hip_device)
    if st != 0:
        raise CropError(st, "crop_create failed")
    return h


def crop_destroy(ctx) -> None:
    _lib.crop_destroy(ctx)


def crop_last_error_detail(ctx) -> str:
    return _lib.crop_last_error_detail(ctx).decode()


def crop_last_error_index(ctx) -> int:
    return _lib.crop_last_error_index(ctx)


def crop_set_partitions(ctx, P: int) -> None:
    _check(ctx, _lib.crop_set_partitions(ctx, P))


def crop_set_seed(ctx, seed: int) -> None:
    _check(ctx, _lib.crop_set_seed(ctx, seed & 0xFFFFFFFFFFFFFFFF))


def crop_set_summary(ctx, counters_per_partition: int, counters_per_bucket: int) -> None:
    _check(ctx, _lib.crop_set_summary(ctx, counters_per_partition, counters_per_bucket))


def crop_set_stream(ctx, stream) -> None:
    """stream: a torch.cuda.Stream or a raw hipStream_t integer (0 or None:
    HIP's null stream)."""
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    _check(ctx, _lib.crop_set_stream(ctx, stream or None))


CROP_RANK_UPPER = 0
CROP_RANK_LOWER = 1


def crop_set_owned_partitions(ctx, p_begin: int, p_end: int) -> None:
    _check(ctx, _lib.crop_set_owned_partitions(ctx, p_begin, p_end))


def crop_set_topk_rank(ctx, rank: int) -> None:
    _check(ctx, _lib.crop_set_topk_rank(ctx, rank))


def crop_use_own_stream(ctx) -> None:
    _check(ctx, _lib.crop_use_own_stream(ctx))


CROP_ROUTE_AUTO = 0
CROP_ROUTE_CHUNKS = 1
CROP_ROUTE_RANGES = 2
CROP_ROUTE_REGIONS = 3
CROP_WINDOW_AUTO = 0
CROP_WINDOW_OFF = 1


def crop_set_tuning(ctx, bins_per_partition=0, rows_per_chunk=0, stage_keys=0,
                    route=CROP_ROUTE_AUTO, window=0, region_terms=0) -> None:
    t = crop_tune(bins_per_partition, rows_per_chunk, stage_keys, route, window, region_terms)
    _check(ctx, _lib.crop_set_tuning(ctx, ctypes.byref(t)))


def crop_autotune(ctx, reps: int = 3):
    """Tune exact runs of the loaded stream; returns (bins_per_partition,
    rows_per_chunk, best_ms) and keeps them as the context's tuning
    (rows_per_chunk is 0 on the region route, whose terms per sub-batch
    crop_get_tuning reports)."""
    S = ctypes.c_uint32(0)
    R = ctypes.c_uint32(0)
    ms = ctypes.c_float(0.0)
    _check(ctx, _lib.crop_autotune(ctx, reps, ctypes.byref(S), ctypes.byref(R), ctypes.byref(ms)))
    return S.value, R.value, float(ms.value)


def crop_get_tuning(ctx) -> dict:
    t = crop_tune()
    _check(ctx, _lib.crop_get_tuning(ctx, ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in crop_tune._fields_}


def crop_load_transactions(ctx, off, items, n_items: int, own: int = CROP_OWN_COPY) -> None:
    """off: uint32[T+1], items: uint32[nnz]; both host (numpy/cpu tensor) or
    both device (cuda tensor)."""
    po, wo = _ptr(off)
    pi, wi = _ptr(items)
    if int(_len(items)) and wo != wi:
        raise ValueError("off and items must both be host or both be device memory")
    _check(ctx, _lib.crop_load_transactions(ctx, po, _len(off) - 1, pi, _len(items), n_items,
                                            wo, own))


def crop_load_outer(ctx, a_off, a_idx, a_val, b_off, b_idx, b_val, n_rows: int, n_cols: int,
                    own: int = CROP_OWN_COPY) -> None:
    ptrs = [_ptr(v) for v in (a_off, a_idx, a_val, b_off, b_idx, b_val)]
    where = ptrs[0][1]
    _check(ctx, _lib.crop_load_outer(ctx, *[p for p, _ in ptrs], _len(a_off) - 1, _len(a_idx),
                                     _len(b_idx), n_rows, n_cols, where, own))


def crop_run_exact(ctx) -> None:
    _check(ctx, _lib.crop_run_exact(ctx))


def crop_run_topk(ctx, K: int) -> None:
    _check(ctx, _lib.crop_run_topk(ctx, K))


def crop_run_topk_seeded(ctx, K: int, sx, sy, r_max: int) -> None:
    px, _ = _ptr(sx)
    py, _ = _ptr(sy)
    _check(ctx, _lib.crop_run_topk_seeded(ctx, K, px, py, _len(sx), r_max))


def crop_run_topk_amplified(ctx, K: int, instances: int, min_votes: int = 0) -> None:
    """Majority reporting over `instances` CRoP runs (seeds seed, seed+1, ...);
    min_votes 0 means at least half: (instances + 1) // 2."""
    if min_votes == 0:
        min_votes = (instances + 1) // 2
    _check(ctx, _lib.crop_run_topk_amplified(ctx, K, instances, min_votes))


def crop_read_topk_votes(ctx, cap: int):
    v = np.zeros(max(cap, 1), np.uint32)
    w = _u64(0)
    _check(ctx, _lib.crop_read_topk_votes(ctx, v.ctypes.data, cap, ctypes.byref(w)))
    return v[:w.value]


def crop_result_sizes(ctx, P: int):
    sizes = np.zeros(P, np.uint64)
    terms = np.zeros(P, np.uint64)
    _check(ctx, _lib.crop_result_sizes(ctx, sizes.ctypes.data, terms.ctypes.data))
    return sizes, terms


def crop_read_partition(ctx, p: int, cap: int, outer: bool = False):
    i = np.zeros(max(cap, 1), np.uint32)
    j = np.zeros(max(cap, 1), np.uint32)
    c = None if outer else np.zeros(max(cap, 1), np.uint32)
    v = np.zeros(max(cap, 1), np.float32) if outer else None
    w = _u64(0)
    _check(ctx, _lib.crop_read_partition(ctx, p, i.ctypes.data, j.ctypes.data,
                                         None if c is None else c.ctypes.data,
                                         None if v is None else v.ctypes.data, cap,
                                         ctypes.byref(w)))
    n = w.value
    return i[:n], j[:n], (v[:n] if outer else c[:n])


def crop_read_all(ctx, P: int, outer: bool = False, device=None):
    """Whole exact result, partition by partition.  With device=None the
    arrays are host numpy arrays; with a torch device they are tensors there."""
    sizes, _ = crop_result_sizes(ctx, P)
    n = int(sizes.sum())
    part_off = np.zeros(P + 1, np.uint64)
    w = _u64(0)
    if device is None:
        i = np.zeros(max(n, 1), np.uint32)
        j = np.zeros(max(n, 1), np.uint32)
        c = None if outer else np.zeros(max(n, 1), np.uint32)
        v = np.zeros(max(n, 1), np.float32) if outer else None
        where = CROP_MEM_HOST
        ptrs = [i.ctypes.data, j.ctypes.data, None if c is None else c.ctypes.data,
                None if v is None else v.ctypes.data]
    else:
        import torch
        i = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        j = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        c = None if outer else torch.empty(max(n, 1), dtype=torch.int32, device=device)
        v = torch.empty(max(n, 1), dtype=torch.float32, device=device) if outer else None
        where = CROP_MEM_DEVICE
        ptrs = [i.data_ptr(), j.data_ptr(), None if c is None else c.data_ptr(),
                None if v is None else v.data_ptr()]
    _check(ctx, _lib.crop_read_all(ctx, where, *ptrs, n, ctypes.byref(w),
                                   part_off.ctypes.data))
    return i[:n], j[:n], (v[:n] if outer else c[:n]), part_off


def crop_read_topk(ctx, cap: int):
    i = np.zeros(max(cap, 1), np.uint32)
    j = np.zeros(max(cap, 1), np.uint32)
    up = np.zeros(max(cap, 1), np.float64)
    lo = np.zeros(max(cap, 1), np.float64)
    val = np.zeros(max(cap, 1), np.float64)
    w = _u64(0)
    _check(ctx, _lib.crop_read_topk(ctx, i.ctypes.data, j.ctypes.data, up.ctypes.data,
                                    lo.ctypes.data, val.ctypes.data, cap, ctypes.byref(w)))
    n = w.value
    return i[:n], j[:n], up[:n], lo[:n], val[:n]


def crop_read_summary(ctx, n_slots: int):
    i = np.zeros(max(n_slots, 1), np.uint32)
    j = np.zeros(max(n_slots, 1), np.uint32)
    cnt = np.zeros(max(n_slots, 1), np.float64)
    err = np.zeros(max(n_slots, 1), np.float64)
    val = np.zeros(max(n_slots, 1), np.float64)
    flags = np.zeros(max(n_slots, 1), np.uint8)
    w = _u64(0)
    _check(ctx, _lib.crop_read_summary(ctx, i.ctypes.data, j.ctypes.data, cnt.ctypes.data,
                                       err.ctypes.data, val.ctypes.data, flags.ctypes.data,
                                       n_slots, ctypes.byref(w)))
    n = w.value
    return dict(x=i[:n], y=j[:n], cnt=cnt[:n], err=err[:n], val=val[:n],
                used=(flags[:n] & 1).astype(bool), pinned=(flags[:n] & 2).astype(bool))


# ---- Count-Sketch

def crop_run_countsketch(ctx, buckets_per_partition: int, instances: int) -> None:
    _check(ctx, _lib.crop_run_countsketch(ctx, buckets_per_partition, instances))


def crop_countsketch_estimate(ctx, qx, qy, est) -> None:
    """qx, qy: uint32/int32 device tensors; est: float64 device tensor."""
    _check(ctx, _lib.crop_countsketch_estimate(ctx, _dev(qx, "qx"), _dev(qy, "qy"), _len(qx),
                                               _dev(est, "est")))


def crop_read_countsketch(ctx, instance: int, n_buckets: int):
    out = np.zeros(max(n_buckets, 1), np.float64)
    _check(ctx, _lib.crop_read_countsketch(ctx, instance, out.ctypes.data, n_buckets))
    return out[:n_buckets]


# ---- batches of transaction streams

def crop_load_batch(ctx, tx_off, off, items, n_items, own: int = CROP_OWN_COPY) -> None:
    """tx_off: uint64[n+1] stream boundaries (host); off, items: the
    concatenated CSR (host arrays or device tensors); n_items: uint32[n]."""
    tx = np.ascontiguousarray(tx_off, np.uint64)
    ni = np.ascontiguousarray(n_items, np.uint32)
    po, wo = _ptr(off)
    pi, wi = _ptr(items)
    if int(_len(items)) and wo != wi:
        raise ValueError("off and items must both be host or both be device memory")
    _check(ctx, _lib.crop_load_batch(ctx, tx.shape[0] - 1, tx.ctypes.data, po, pi, ni.ctypes.data,
                                     wo, own))


def crop_batch_set_plan(ctx, terms_per_bin: int, rows_per_chunk: int) -> None:
    _check(ctx, _lib.crop_batch_set_plan(ctx, terms_per_bin, rows_per_chunk))


def crop_batch_autotune(ctx, reps: int = 2):
    """(terms_per_bin, rows_per_chunk, best ms) of the fastest candidate."""
    t, r, ms = _u32(0), _u32(0), ctypes.c_float(0.0)
    _check(ctx, _lib.crop_batch_autotune(ctx, reps, ctypes.byref(t), ctypes.byref(r),
                                         ctypes.byref(ms)))
    return t.value, r.value, float(ms.value)


def crop_batch_set_graph(ctx, enable: bool) -> None:
    _check(ctx, _lib.crop_batch_set_graph(ctx, 1 if enable else 0))


def crop_run_exact_batched(ctx) -> None:
    _check(ctx, _lib.crop_run_exact_batched(ctx))


def crop_batch_info(ctx, stream: int) -> dict:
    p, t, f, n = _u32(0), _u64(0), _u64(0), _u64(0)
    _check(ctx, _lib.crop_batch_info(ctx, stream, ctypes.byref(p), ctypes.byref(t),
                                     ctypes.byref(f), ctypes.byref(n)))
    return dict(partitions=p.value, terms=t.value, first_tx=f.value, n_tx=n.value)


def crop_batch_result_sizes(ctx, stream: int):
    P = crop_batch_info(ctx, stream)["partitions"]
    sizes = np.zeros(max(P, 1), np.uint64)
    terms = np.zeros(max(P, 1), np.uint64)
    _check(ctx, _lib.crop_batch_result_sizes(ctx, stream, sizes.ctypes.data, terms.ctypes.data))
    return sizes[:P], terms[:P]


def crop_batch_read_stream(ctx, stream: int):
    """(i, j, count, part_off) of stream `stream` as host arrays."""
    sizes, _ = crop_batch_result_sizes(ctx, stream)
    n = int(sizes.sum())
    P = sizes.shape[0]
    i = np.zeros(max(n, 1), np.uint32)
    j = np.zeros(max(n, 1), np.uint32)
    c = np.zeros(max(n, 1), np.uint32)
    part_off = np.zeros(P + 1, np.uint64)
    w = _u64(0)
    _check(ctx, _lib.crop_batch_read_stream(ctx, stream, CROP_MEM_HOST, i.ctypes.data,
                                            j.ctypes.data, c.ctypes.data, n, ctypes.byref(w),
                                            part_off.ctypes.data))
    return i[:n], j[:n], c[:n], part_off


# ---- learned heavy-pair seeding (device tensors in and out)

MLP_PARAMS = 6337


def _dev(a, name):
    p, where = _ptr(a)
    if a is not None and where != CROP_MEM_DEVICE:
        raise ValueError(f"{name} must be device memory")
    return p


def crop_item_features(ctx, prefix_T: int, feat) -> None:
    """feat: float32 device tensor [n_items, 16]."""
    _check(ctx, _lib.crop_item_features(ctx, prefix_T, _dev(feat, "feat")))


def crop_item_features_noalloc(ctx, prefix_T: int, feat) -> None:
    """crop_item_features with the library's fixed per-GPU workspace (no
    allocation); feat: float32 device tensor [n_items, 16]."""
    _check(ctx, _lib.crop_item_features_noalloc(ctx, prefix_T, _dev(feat, "feat")))


def crop_top_item_pairs(ctx, prefix_T: int, M: int, cx, cy) -> int:
    """cx, cy: uint32/int32 device tensors of capacity >= M(M-1)/2."""
    n = _u64(0)
    _check(ctx, _lib.crop_top_item_pairs(ctx, prefix_T, M, _dev(cx, "cx"), _dev(cy, "cy"),
                                         _len(cx), ctypes.byref(n)))
    return n.value


def crop_lookup_exact(ctx, qx, qy, count) -> None:
    _check(ctx, _lib.crop_lookup_exact(ctx, _dev(qx, "qx"), _dev(qy, "qy"), _len(qx),
                                       _dev(count, "count")))


def crop_pair_inputs(ctx, feat, cx, cy, count, Z, y=None) -> None:
    _check(ctx, _lib.crop_pair_inputs(ctx, _dev(feat, "feat"), _dev(cx, "cx"), _dev(cy, "cy"),
                                      _dev(count, "count"), _len(cx), _dev(Z, "Z"),
                                      _dev(y, "y")))


def crop_mlp_create(ctx, init):
    """init: float32 host array of MLP_PARAMS values."""
    init = np.ascontiguousarray(init, np.float32)
    if init.shape != (MLP_PARAMS,):
        raise ValueError(f"init must hold {MLP_PARAMS} floats")
    h = _vp()
    _check(ctx, _lib.crop_mlp_create(ctx, init.ctypes.data, ctypes.byref(h)))
    return h


def crop_mlp_destroy(mlp) -> None:
    _lib.crop_mlp_destroy(mlp)


def crop_mlp_params(ctx, mlp):
    out = np.zeros(MLP_PARAMS, np.float32)
    _check(ctx, _lib.crop_mlp_params(ctx, mlp, out.ctypes.data))
    return out


def crop_mlp_grad(ctx, mlp, Z, y):
    """(gradient [MLP_PARAMS], loss) of the MSE over the samples Z, y."""
    g = np.zeros(MLP_PARAMS, np.float32)
    loss = ctypes.c_float(0.0)
    _check(ctx, _lib.crop_mlp_grad(ctx, mlp, _dev(Z, "Z"), _dev(y, "y"), _len(y),
                                   g.ctypes.data, ctypes.byref(loss)))
    return g, float(loss.value)


def crop_mlp_train(ctx, mlp, Z, y, order, batch: int, lr: float) -> None:
    _check(ctx, _lib.crop_mlp_train(ctx, mlp, _dev(Z, "Z"), _dev(y, "y"), _len(y),
                                    _dev(order, "order"), _len(order), batch, lr))


def crop_mlp_loss(ctx, mlp) -> float:
    loss = ctypes.c_float(0.0)
    _check(ctx, _lib.crop_mlp_loss(ctx, mlp, ctypes.byref(loss)))
    return float(loss.value)


def crop_mlp_score(ctx, mlp, Z, out) -> None:
    _check(ctx, _lib.crop_mlp_score(ctx, mlp, _dev(Z, "Z"), _len(out), _dev(out, "out")))


def crop_select_seeds(ctx, score, cx, cy, R: int, sx, sy) -> None:
    _check(ctx, _lib.crop_select_seeds(ctx, _dev(score, "score"), _dev(cx, "cx"),
                                       _dev(cy, "cy"), _len(score), R, _dev(sx, "sx"),
                                       _dev(sy, "sy")))


def crop_hash_pairs(ctx, qx, qy, h=None, part=None) -> None:
    """h[q], part[q] of the pairs (qx[q], qy[q]); device tensors, either
    output may be None."""
    _check(ctx, _lib.crop_hash_pairs(ctx, _dev(qx, "qx"), _dev(qy, "qy"), _len(qx),
                                     _dev(h, "h"), _dev(part, "part")))


def crop_predictor_train(ctx, streams, top_items: int = 0, epochs: int = 0, batch: int = 0,
                         lr: float = 0.0, shuffle_seed: int = 0, init=None):
    """Train a predictor on `streams`, a list of (off, items, n_items) with the
    arrays all numpy (host) or all torch device tensors; returns the handle."""
    refs = (crop_stream_ref * len(streams))()
    where = None
    keep = []
    for k, (off, items, n) in enumerate(streams):
        po, wo = _ptr(off)
        pi, wi = _ptr(items)
        if where is None:
            where = wo
        if wo != where or (len(items) and wi != where):
            raise ValueError("every training array must be host or every one device")
        keep += [off, items]
        refs[k] = crop_stream_ref(po, _len(off) - 1, pi, _len(items), int(n))
    tset = crop_train_set(refs, len(streams), CROP_MEM_HOST if where is None else where)
    w = None if init is None else np.ascontiguousarray(init, np.float32)
    opts = crop_train_opts(top_items, epochs, batch, lr, shuffle_seed,
                           None if w is None else w.ctypes.data)
    out = _vp()
    _check(ctx, _lib.crop_predictor_train(ctx, ctypes.byref(tset), ctypes.byref(opts),
                                          ctypes.byref(out)))
    return out.value


def crop_predictor_score(ctx, pred, R: int, sx, sy) -> int:
    """Seeds of the loaded stream into device tensors sx, sy (capacity R);
    returns how many were written."""
    n = _u64(0)
    _check(ctx, _lib.crop_predictor_score(ctx, pred, R, _dev(sx, "sx"), _dev(sy, "sy"),
                                          ctypes.byref(n)))
    return int(n.value)


def crop_predictor_params(ctx, pred):
    """(weights [MLP_PARAMS], mean loss of the last training minibatch)."""
    out = np.zeros(MLP_PARAMS, np.float32)
    loss = ctypes.c_float(0.0)
    _check(ctx, _lib.crop_predictor_params(ctx, pred, out.ctypes.data, ctypes.byref(loss)))
    return out, float(loss.value)


def crop_predictor_free(pred) -> None:
    _lib.crop_predictor_free(pred)


def crop_synchronize(ctx) -> None:
    _check(ctx, _lib.crop_synchronize(ctx))


def crop_last_run_ms(ctx) -> float:
    ms = ctypes.c_float(0.0)
    _check(ctx, _lib.crop_last_run_ms(ctx, ctypes.byref(ms)))
    return float(ms.value)


def crop_set_profiling(ctx, enable: bool) -> None:
    _check(ctx, _lib.crop_set_profiling(ctx, 1 if enable else 0))


def crop_run_stages(ctx, back: int = 0):
    """[(stage name, device ms)] of the run `back` runs ago (profiling on)."""
    cap = 16
    n = _u32(0)
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_float * cap)()
    _check(ctx, _lib.crop_run_stages(ctx, back, ctypes.byref(n), names, ms, cap))
    return [(names[k].decode(), float(ms[k])) for k in range(n.value)]


def _len(a) -> int:
    return int(a.shape[0]) if hasattr(a, "shape") else len(a)
