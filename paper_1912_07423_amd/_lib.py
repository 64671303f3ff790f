"""ctypes declarations of the C ABI in include/snn.h and the loader of libsnn.so.

The library is built in-tree (``python -m paper_1912_07423_amd.build`` or
``__graft_entry__.build()``).  Loading fails loudly if it is missing: there is no
fallback path.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsnn.so")

SNN_OK = 0
SNN_E_INVALID = -1
SNN_E_OOM = -2
SNN_E_HIP = -3
SNN_E_OVERFLOW = -4
SNN_E_STATE = -5
STATUS_NAMES = {0: "SNN_OK", -1: "SNN_E_INVALID", -2: "SNN_E_OOM", -3: "SNN_E_HIP",
                -4: "SNN_E_OVERFLOW", -5: "SNN_E_STATE"}

PROJ_KIND = {"er": 0, "fixed": 1}
DELIVERY = {"auto": 0, "atomic": 1, "tiled": 2}
PLASTICITY = {"eager": 0, "lazy": 1}
DELIVERY_NAME = {1: "atomic", 2: "tiled"}


class Population(C.Structure):
    _fields_ = [("size", C.c_uint32), ("excitatory", C.c_uint32)]


class Projection(C.Structure):
    _fields_ = [("from_", C.c_uint32), ("to", C.c_uint32), ("kind", C.c_uint32), ("k", C.c_uint32),
                ("p", C.c_double), ("w_mV", C.c_double), ("plastic", C.c_uint32),
                ("to_span", C.c_uint32)]


PARAM_FIELDS = [
    ("dt_ms", C.c_double), ("delay_steps", C.c_uint32), ("n_ext", C.c_uint32),
    ("tau_m_ms", C.c_double), ("v_rest_mV", C.c_double), ("v_bg_mV", C.c_double),
    ("v_th_mV", C.c_double), ("v_reset_mV", C.c_double), ("t_ref_ms", C.c_double),
    ("v0_lo_mV", C.c_double), ("v0_hi_mV", C.c_double), ("rate_ext_hz", C.c_double),
    ("w_ext_mV", C.c_double), ("tau_plus_ms", C.c_double), ("tau_minus_ms", C.c_double),
    ("a_plus", C.c_double), ("a_minus", C.c_double), ("w_max_mV", C.c_double),
    ("seed", C.c_uint64), ("raster_steps", C.c_uint32), ("window", C.c_uint32),
    ("delivery", C.c_uint32), ("tiles", C.c_uint32), ("block", C.c_uint32),
    ("grid", C.c_uint32), ("synapse_weights", C.c_uint32), ("plasticity", C.c_uint32),
]


class Params(C.Structure):
    _fields_ = PARAM_FIELDS


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("n", C.c_uint32), ("delay", C.c_uint32), ("queue_slots", C.c_uint32),
                ("input_buffers", C.c_uint32), ("window", C.c_uint32), ("delivery", C.c_uint32),
                ("tiles", C.c_uint32), ("plastic", C.c_uint32), ("raster_steps", C.c_uint32),
                ("raster_words", C.c_uint32), ("table_len", C.c_uint32),
                ("queue_groups", C.c_uint32), ("queue_stride", C.c_uint32),
                ("source_weights", C.c_uint32),
                ("nnz", C.c_uint64), ("t", C.c_uint64), ("events", C.c_uint64),
                ("spikes", C.c_uint64), ("touches", C.c_uint64), ("device_bytes", C.c_uint64),
                ("build_ms", C.c_double), ("gen_rows_ms", C.c_float), ("gen_fill_ms", C.c_float),
                ("index_ms", C.c_float), ("tile_offset_bytes", C.c_uint32),
                ("target_bytes", C.c_uint32), ("plasticity", C.c_uint32)]


class State(C.Structure):
    _fields_ = [("v", C.c_void_p), ("ref", C.c_void_p), ("input", C.c_void_p),
                ("x_pre", C.c_void_p), ("x_post", C.c_void_p), ("queue", C.c_void_p),
                ("queue_len", C.c_void_p), ("w_f32", C.c_void_p)]


class Profile(C.Structure):
    _fields_ = [("update_ms", C.c_double), ("deliver_ms", C.c_double), ("stdp_ms", C.c_double),
                ("update_launches", C.c_uint64), ("deliver_launches", C.c_uint64),
                ("stdp_launches", C.c_uint64)]


class DeliveryTuning(C.Structure):
    _fields_ = [("delivery", C.c_uint32), ("tiles", C.c_uint32), ("block", C.c_uint32),
                ("grid", C.c_uint32), ("ms_per_launch", C.c_double), ("events_per_launch", C.c_uint64)]


class BatchMember(C.Structure):
    _fields_ = [("params", C.POINTER(Params)), ("pops", C.POINTER(Population)),
                ("proj", C.POINTER(Projection)), ("n_pops", C.c_uint32), ("n_proj", C.c_uint32)]


class BatchTuning(C.Structure):
    _fields_ = [("block", C.c_uint32), ("per_lane", C.c_uint32), ("degree_div", C.c_uint32),
                ("pad_", C.c_uint32), ("ms_per_step", C.c_double)]


class BpttDesc(C.Structure):
    _fields_ = [("batch", C.c_uint32), ("steps", C.c_uint32), ("n_in", C.c_uint32),
                ("n_hidden", C.c_uint32), ("n_out", C.c_uint32), ("checkpoint", C.c_uint32),
                ("beta", C.c_float), ("beta_out", C.c_float), ("theta", C.c_float),
                ("slope", C.c_float), ("smooth", C.c_uint32), ("eager", C.c_uint32)]


# every symbol declared in include/snn.h, with its ctypes signature
SIGNATURES = {
    "snn_build_network": (C.c_int32, [C.POINTER(Params), C.POINTER(Population), C.c_uint32,
                                      C.POINTER(Projection), C.c_uint32, C.POINTER(Allocator),
                                      C.c_void_p, C.POINTER(C.c_void_p)]),
    "snn_step": (C.c_int32, [C.c_void_p]),
    "snn_run": (C.c_int32, [C.c_void_p, C.c_uint32]),
    "snn_get_raster": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p,
                                   C.c_uint64, C.POINTER(C.c_uint64)]),
    "snn_get_raster_bits": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p]),
    "snn_get_info": (C.c_int32, [C.c_void_p, C.POINTER(Info)]),
    "snn_get_state": (C.c_int32, [C.c_void_p, C.POINTER(State)]),
    "snn_set_state": (C.c_int32, [C.c_void_p, C.POINTER(State)]),
    "snn_get_row": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_uint64, C.POINTER(C.c_uint64)]),
    "snn_get_synapses": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "snn_get_drive_table": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint32]),
    "snn_spacing_gaps": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]),
    "snn_set_profiling": (C.c_int32, [C.c_void_p, C.c_int32]),
    "snn_get_profile": (C.c_int32, [C.c_void_p, C.POINTER(Profile)]),
    "snn_reset_profile": (C.c_int32, [C.c_void_p]),
    "snn_sync": (C.c_int32, [C.c_void_p]),
    "snn_memory_cache_stats": (C.c_int32, [C.c_int, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                           C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "snn_memory_cache_release": (C.c_int32, [C.c_int]),
    "snn_time_delivery": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32, C.c_uint32,
                                      C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    "snn_time_delivery_static": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32,
                                             C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    "snn_set_delivery": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]),
    "snn_autotune_delivery": (C.c_int32, [C.c_void_p, C.c_uint32, C.POINTER(DeliveryTuning)]),
    "snn_destroy": (None, [C.c_void_p]),
    "snn_last_error": (C.c_char_p, [C.c_void_p]),
    "snn_build_batch": (C.c_int32, [C.POINTER(BatchMember), C.c_uint32, C.c_uint32,
                                    C.POINTER(Allocator), C.c_void_p, C.POINTER(C.c_void_p)]),
    "snn_batch_run": (C.c_int32, [C.c_void_p, C.c_uint32]),
    "snn_batch_sync": (C.c_int32, [C.c_void_p]),
    "snn_batch_network": (C.c_int32, [C.c_void_p, C.c_uint32, C.POINTER(C.c_void_p)]),
    "snn_batch_autotune": (C.c_int32, [C.c_void_p, C.c_uint32, C.POINTER(BatchTuning)]),
    "snn_batch_set_tuning": (C.c_int32, [C.c_void_p, C.POINTER(BatchTuning)]),
    "snn_batch_get_tuning": (C.c_int32, [C.c_void_p, C.POINTER(BatchTuning)]),
    "snn_batch_destroy": (None, [C.c_void_p]),
    "snn_bptt_create": (C.c_int32, [C.POINTER(BpttDesc), C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.POINTER(Allocator), C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "snn_bptt_forward": (C.c_int32, [C.c_void_p] + [C.c_void_p] * 6 + [C.c_void_p]),
    "snn_bptt_backward": (C.c_int32, [C.c_void_p] + [C.c_void_p] * 7 + [C.c_void_p]),
    "snn_bptt_get_trace": (C.c_int32, [C.c_void_p] + [C.c_void_p] * 4 + [C.c_void_p]),
    "snn_bptt_destroy": (None, [C.c_void_p]),
}

_lib = None


class SnnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load():
    """The loaded library; raises if it has not been built.  PyTorch, when installed, is
    imported first, so that the process has one HIP runtime: the one torch brings, which
    libsnn.so then binds to, whatever order the caller imports things in."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1912_07423_amd.build` (hipcc, gfx950)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status):
    if status != SNN_OK:
        raise SnnError(status, load().snn_last_error(None).decode(errors="replace"))
