"""ctypes view of include/relnn.h.  Loads the in-tree librelnn.so and fails
loudly when it is missing: there is no fallback path."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librelnn.so")

OK, E_INVALID, E_RANGE, E_NOT_UNIQUE, E_OOM, E_HIP, E_BUSY, E_NOT_READY, E_UNSUPPORTED = range(9)
STATUS_NAMES = ["OK", "INVALID", "RANGE", "NOT_UNIQUE", "OOM", "HIP", "BUSY", "NOT_READY",
                "UNSUPPORTED"]
F32, BF16 = 0, 1
SUM, MEAN, MAX = 0, 1, 2
ACT_NONE, ACT_RELU = 0, 1
IDX_BWD = 1
FUSED, PLAIN, DW_ACCUM, OUT_BF16, PUSHDOWN, TF_PRODUCT = 0, 1, 2, 4, 8, 16
MAX_ATOMS = 4

p_i32 = C.POINTER(C.c_int32)


class Atom(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("keys", C.c_void_p), ("col", C.c_int32)]


class Chain(C.Structure):
    _fields_ = [("src_col", C.c_int32), ("n_rows", C.c_int64), ("keys", C.c_void_p),
                ("vals", C.c_void_p)]


class JoinStep(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("n_cols", C.c_int32), ("cols", C.POINTER(C.c_void_p)),
                ("n_on", C.c_int32), ("on", C.c_int32 * 2), ("key", C.c_int32 * 2)]


class Pred(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32), ("mul_a", C.c_int64), ("mul_b", C.c_int64),
                ("add", C.c_int64), ("op", C.c_int32)]


CMP = {"eq": 0, "ne": 1, "lt": 2, "le": 3, "gt": 4, "ge": 5}


class AttnDesc(C.Structure):
    _fields_ = [("heads", C.c_int32), ("d", C.c_int32), ("dv", C.c_int32), ("scale", C.c_float),
                ("dtype", C.c_int32)]


class JoinDesc(C.Structure):
    _fields_ = [("n_link", C.c_int64), ("n_cols", C.c_int32), ("cols", C.POINTER(C.c_void_p)),
                ("n_chains", C.c_int32), ("chains", C.POINTER(Chain)),
                ("n_atoms", C.c_int32), ("atoms", C.POINTER(Atom)),
                ("group_col", C.c_int32), ("two_hop_mid", C.c_int32), ("two_hop_cap", C.c_int32),
                ("flags", C.c_uint32), ("n_steps", C.c_int32), ("steps", C.POINTER(JoinStep)),
                ("n_preds", C.c_int32), ("preds", C.POINTER(Pred))]


class LayerDesc(C.Structure):
    _fields_ = [("k", C.c_int32), ("d", p_i32), ("h", C.c_int32), ("dtype", C.c_int32),
                ("agg", C.c_int32), ("act_pre", C.c_int32), ("act_post", C.c_int32),
                ("flags", C.c_uint32)]


class ServeDesc(C.Structure):
    _fields_ = [("n_user", C.c_int64), ("n_item", C.c_int64), ("n_cat", C.c_int64), ("n_buys", C.c_int64),
                ("buys_user", C.c_void_p), ("buys_item", C.c_void_p), ("item_cat", C.c_void_p),
                ("user_emb", C.c_void_p), ("item_emb", C.c_void_p), ("cat_emb", C.c_void_p),
                ("d", C.c_int32), ("h", C.c_int32),
                ("W_user", C.c_void_p), ("W_item1", C.c_void_p), ("W_item2", C.c_void_p),
                ("b_user", C.c_void_p), ("b_item1", C.c_void_p), ("b_item2", C.c_void_p),
                ("fanout1", C.c_int32), ("fanout2", C.c_int32), ("dtype", C.c_int32),
                ("max_seeds", C.c_int32), ("max_slots", C.c_int32), ("budget_bytes", C.c_size_t)]


class ReqStats(C.Structure):
    _fields_ = [("t_arrive_ns", C.c_int64), ("t_admit_ns", C.c_int64), ("t_done_ns", C.c_int64),
                ("tuples", C.c_int64), ("step", C.c_int64), ("n_seeds", C.c_int32)]


class RelnnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"relnn error {name}: {msg}")
        self.status = status


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "relnn_build_index": (C.c_int, [C.POINTER(JoinDesc), C.c_void_p, C.POINTER(C.c_void_p)]),
    "relnn_index_query": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64)]),
    "relnn_index_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "relnn_index_free": (C.c_int, [C.c_void_p]),
    "relnn_workspace_size": (C.c_int, [C.c_void_p, C.POINTER(LayerDesc), C.c_int, C.POINTER(C.c_size_t)]),
    "relnn_layer_fwd": (C.c_int, [C.c_void_p, C.POINTER(LayerDesc), C.POINTER(C.c_void_p), C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                  C.c_void_p]),
    "relnn_layer_fwd_static": (C.c_int, [C.c_void_p, C.POINTER(LayerDesc), C.POINTER(C.c_void_p), C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "relnn_static_scratch_bytes": (C.c_int, [C.POINTER(C.c_size_t)]),
    "relnn_attn_workspace_size": (C.c_int, [C.c_void_p, C.POINTER(AttnDesc), C.c_int, C.POINTER(C.c_size_t)]),
    "relnn_attn_fwd": (C.c_int, [C.c_void_p, C.POINTER(AttnDesc), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "relnn_attn_bwd": (C.c_int, [C.c_void_p, C.POINTER(AttnDesc), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_size_t, C.c_void_p]),
    "relnn_out_dense": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "relnn_union_build": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "relnn_union_query": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "relnn_union_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "relnn_union_free": (C.c_int, [C.c_void_p]),
    "relnn_union_workspace_size": (C.c_int, [C.c_void_p, C.POINTER(C.POINTER(LayerDesc)), C.c_int32,
                                             C.POINTER(C.c_size_t)]),
    "relnn_union_fwd": (C.c_int, [C.c_void_p, C.POINTER(C.POINTER(LayerDesc)), C.c_int32, C.c_int32,
                                  C.POINTER(C.POINTER(C.c_void_p)), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_size_t, C.c_void_p]),
    "relnn_union_bwd_workspace_size": (C.c_int, [C.c_void_p, C.POINTER(C.POINTER(LayerDesc)), C.c_int32, C.c_int32,
                                                 C.POINTER(C.c_size_t)]),
    "relnn_union_bwd": (C.c_int, [C.c_void_p, C.POINTER(C.POINTER(LayerDesc)), C.c_int32, C.c_int32,
                                  C.POINTER(C.POINTER(C.c_void_p)), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.POINTER(C.POINTER(C.c_void_p)), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "relnn_layer_bwd": (C.c_int, [C.c_void_p, C.POINTER(LayerDesc), C.POINTER(C.c_void_p), C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p),
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "relnn_serve_create": (C.c_int, [C.POINTER(ServeDesc), C.POINTER(C.c_void_p)]),
    "relnn_serve_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_uint64, C.POINTER(C.c_uint64)]),
    "relnn_serve_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.POINTER(ReqStats)]),
    "relnn_serve_cancel": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32)]),
    "relnn_serve_destroy": (C.c_int, [C.c_void_p]),
    "relnn_timing_enable": (C.c_int, [C.c_int]),
    "relnn_timing_reset": (C.c_int, []),
    "relnn_timing_read": (C.c_int, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "relnn_last_error": (C.c_char_p, []),
}

OPTIONAL = set()


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2605_24207_amd.build` "
                              "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            if not hasattr(L, name):
                if name in OPTIONAL:
                    continue
                raise ImportError(f"{LIB_PATH} does not export {name}")
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != OK:
        raise RelnnError(status, lib().relnn_last_error().decode(errors="replace"))


def exported_symbols():
    return sorted(_SIGS)
