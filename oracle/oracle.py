"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use this
module.  It never imports the GPU package; workloads are passed in as plain dicts:

    spec = {"params": {...orc_params fields...},
            "pops":   [{"size": int, "excitatory": 0|1}, ...],
            "projs":  [{"from": a, "to": b, "kind": "er"|"fixed", "p": float,
                        "k": int, "w_mV": float, "plastic": 0|1}, ...]}
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class Pop(C.Structure):
    _fields_ = [("size", C.c_uint32), ("excitatory", C.c_uint32)]


class Proj(C.Structure):
    _fields_ = [("from_", C.c_uint32), ("to", C.c_uint32), ("kind", C.c_uint32),
                ("k", C.c_uint32), ("p", C.c_double), ("w_mV", C.c_double),
                ("plastic", C.c_uint32), ("to_span", C.c_uint32)]


PARAM_FIELDS = [
    ("dt_ms", C.c_double), ("delay_steps", C.c_uint32), ("n_ext", C.c_uint32),
    ("tau_m_ms", C.c_double), ("v_rest_mV", C.c_double), ("v_bg_mV", C.c_double),
    ("v_th_mV", C.c_double), ("v_reset_mV", C.c_double), ("t_ref_ms", C.c_double),
    ("v0_lo_mV", C.c_double), ("v0_hi_mV", C.c_double),
    ("rate_ext_hz", C.c_double), ("w_ext_mV", C.c_double),
    ("tau_plus_ms", C.c_double), ("tau_minus_ms", C.c_double), ("a_plus", C.c_double),
    ("a_minus", C.c_double), ("w_max_mV", C.c_double), ("seed", C.c_uint64),
]


class Params(C.Structure):
    _fields_ = PARAM_FIELDS


class View(C.Structure):
    _fields_ = [
        ("n", C.c_uint32), ("delay", C.c_uint32), ("n_slots", C.c_uint32),
        ("raster_cap", C.c_uint32), ("raster_words", C.c_uint32), ("plastic", C.c_uint32),
        ("table_len", C.c_uint32), ("pad_", C.c_uint32),
        ("nnz", C.c_uint64), ("t", C.c_uint64), ("events", C.c_uint64), ("touches", C.c_uint64),
        ("v", C.POINTER(C.c_float)), ("x_pre", C.POINTER(C.c_float)),
        ("x_post", C.POINTER(C.c_float)), ("w_f32", C.POINTER(C.c_float)),
        ("ref", C.POINTER(C.c_int32)), ("input", C.POINTER(C.c_int32)),
        ("col", C.POINTER(C.c_int32)), ("w_q16", C.POINTER(C.c_int32)),
        ("row_ptr", C.POINTER(C.c_uint64)), ("raster", C.POINTER(C.c_uint64)),
        ("table", C.POINTER(C.c_uint64)),
        ("queue_len", C.POINTER(C.c_uint32)), ("queue", C.POINTER(C.c_int32)),
        ("alpha", C.c_float), ("v_inf", C.c_float), ("v_th", C.c_float),
        ("v_reset", C.c_float), ("beta_plus", C.c_float), ("beta_minus", C.c_float),
        ("a_plus", C.c_float), ("a_minus", C.c_float), ("w_max", C.c_float),
        ("ref_steps", C.c_int32), ("w_ext_q16", C.c_int32),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        u32p = C.POINTER(C.c_uint32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_neg_log.argtypes = [C.c_double]
        L.orc_neg_log.restype = C.c_double
        L.orc_spacing_core.argtypes = [C.POINTER(C.c_double), C.c_uint32, C.c_uint64,
                                       C.POINTER(C.c_uint64), C.POINTER(C.c_int64)]
        L.orc_binom_table.argtypes = [C.c_uint32, C.c_double, C.POINTER(C.c_uint64), C.c_uint32]
        L.orc_binom_table.restype = C.c_uint32
        L.orc_gen_row.argtypes = [C.POINTER(Params), C.POINTER(Pop), C.c_uint32,
                                  C.POINTER(Proj), C.c_uint32, C.c_uint32,
                                  C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_float), C.c_int64]
        L.orc_gen_row.restype = C.c_int64
        L.orc_create.argtypes = [C.POINTER(Params), C.POINTER(Pop), C.c_uint32,
                                 C.POINTER(Proj), C.c_uint32, C.c_uint32, C.c_char_p,
                                 C.c_size_t]
        L.orc_create.restype = C.c_void_p
        L.orc_create_neurons_only.argtypes = [C.POINTER(Params), C.POINTER(Pop), C.c_uint32,
                                              C.c_char_p, C.c_size_t]
        L.orc_create_neurons_only.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_view_get.argtypes = [C.c_void_p, C.POINTER(View)]
        L.orc_run.argtypes = [C.c_void_p, C.c_uint32]
        L.orc_update_range.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32,
                                       C.POINTER(C.c_float), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_uint64)]
        L.orc_update_range.restype = C.c_uint32
        L.orc_deliver_generated.argtypes = [C.POINTER(Params), C.POINTER(Pop), C.c_uint32,
                                            C.POINTER(Proj), C.c_uint32,
                                            C.POINTER(C.c_uint32), C.c_uint32,
                                            C.POINTER(C.c_int32)]
        L.orc_deliver_generated.restype = C.c_uint64
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def neg_log(u: float) -> float:
    return lib().orc_neg_log(float(u))


def spacing_core(u, spare: int):
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = len(u) - 1
    S = np.zeros(n + 2, dtype=np.uint64)
    x = np.zeros(max(n, 1), dtype=np.int64)
    lib().orc_spacing_core(_ptr(u, C.c_double), n, spare, _ptr(S, C.c_uint64), _ptr(x, C.c_int64))
    return S, x[:n]


def binom_table(n: int, p: float, cap: int = 256):
    t = np.zeros(cap, dtype=np.uint64)
    m = lib().orc_binom_table(n, p, _ptr(t, C.c_uint64), cap)
    return t[:m]


def _structs(spec):
    prm = Params(**{k: spec["params"][k] for k, _ in PARAM_FIELDS})
    pops = (Pop * len(spec["pops"]))(*[Pop(p["size"], p.get("excitatory", 1)) for p in spec["pops"]])
    projs = spec.get("projs", [])
    kinds = {"er": 0, "fixed": 1}
    arr = (Proj * max(1, len(projs)))()
    for q, pj in enumerate(projs):
        arr[q] = Proj(pj["from"], pj["to"], kinds[pj["kind"]], int(pj.get("k", 0)),
                      float(pj.get("p", 0.0)), float(pj["w_mV"]), int(pj.get("plastic", 0)),
                      int(pj.get("to_span", 1)))
    return prm, pops, len(spec["pops"]), arr, len(projs)


def gen_row(spec, i: int, cap: int = 1 << 20):
    prm, pops, npop, projs, nproj = _structs(spec)
    col = np.zeros(cap, dtype=np.int32)
    wq = np.zeros(cap, dtype=np.int32)
    wf = np.zeros(cap, dtype=np.float32)
    n = lib().orc_gen_row(C.byref(prm), pops, npop, projs, nproj, i, _ptr(col, C.c_int32),
                          _ptr(wq, C.c_int32), _ptr(wf, C.c_float), cap)
    if n < 0:
        raise ValueError("orc_gen_row failed")
    return col[:n].copy(), wq[:n].copy(), wf[:n].copy()


def deliver_generated(spec, spikes, n_neurons: int):
    """Input accumulators (int32) after delivering the given spike list into zeros."""
    prm, pops, npop, projs, nproj = _structs(spec)
    s = np.ascontiguousarray(spikes, dtype=np.uint32)
    inp = np.zeros(n_neurons, dtype=np.int32)
    ev = lib().orc_deliver_generated(C.byref(prm), pops, npop, projs, nproj,
                                     _ptr(s, C.c_uint32), len(s), _ptr(inp, C.c_int32))
    if ev == (1 << 64) - 1:
        raise ValueError("invalid spec")
    return inp, int(ev)


class OracleNet:
    """A whole network simulated step by step on the CPU."""

    def __init__(self, spec, raster_cap: int = 1, neurons_only: bool = False):
        prm, pops, npop, projs, nproj = _structs(spec)
        err = C.create_string_buffer(256)
        if neurons_only:
            h = lib().orc_create_neurons_only(C.byref(prm), pops, npop, err, 256)
        else:
            h = lib().orc_create(C.byref(prm), pops, npop, projs, nproj, raster_cap, err, 256)
        if not h:
            raise ValueError("oracle rejected the network: " + err.value.decode())
        self._h = h
        self._refresh()

    def _refresh(self):
        v = View()
        lib().orc_view_get(self._h, C.byref(v))
        self._v = v

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, n_steps: int):
        lib().orc_run(self._h, n_steps)
        self._refresh()

    def _arr(self, name, n, dtype):
        p = getattr(self._v, name)
        if not p or n == 0:
            return np.zeros(0, dtype=dtype)
        return np.ctypeslib.as_array(p, shape=(n,))

    # live views into oracle memory (writes change the oracle state)
    @property
    def n(self):
        return self._v.n

    @property
    def t(self):
        self._refresh()
        return self._v.t

    @property
    def events(self):
        self._refresh()
        return self._v.events

    @property
    def touches(self):
        self._refresh()
        return self._v.touches

    @property
    def nnz(self):
        return self._v.nnz

    @property
    def const(self):
        return self._v

    def v(self):
        return self._arr("v", self.n, np.float32)

    def ref(self):
        return self._arr("ref", self.n, np.int32)

    def input(self):
        return self._arr("input", self.n, np.int32)

    def x_pre(self):
        return self._arr("x_pre", self.n, np.float32)

    def x_post(self):
        return self._arr("x_post", self.n, np.float32)

    def row_ptr(self):
        return self._arr("row_ptr", self.n + 1, np.uint64)

    def col(self):
        return self._arr("col", self.nnz, np.int32)

    def w_q16(self):
        return self._arr("w_q16", self.nnz, np.int32)

    def w_f32(self):
        return self._arr("w_f32", self.nnz, np.float32)

    def table(self):
        return self._arr("table", self._v.table_len, np.uint64)

    def raster_words(self):
        """[raster_cap, words] uint64 bitmask ring; row t % raster_cap holds step t."""
        v = self._v
        a = self._arr("raster", v.raster_cap * v.raster_words, np.uint64)
        return a.reshape(v.raster_cap, v.raster_words)

    def raster_bool(self, t0: int, t1: int):
        """Spike matrix [t1 - t0, n] for steps in [t0, t1) still held by the ring."""
        v = self._v
        words = self.raster_words()
        rows = np.stack([words[t % v.raster_cap] for t in range(t0, t1)]) if t1 > t0 else \
            np.zeros((0, v.raster_words), dtype=np.uint64)
        bits = np.unpackbits(rows.view(np.uint8), axis=1, bitorder="little")
        return bits[:, : self.n].astype(bool)

    def update_range(self, t: int, v, ref, inp):
        """One neuron update of step t on caller arrays (neuron constants of this net)."""
        n = len(v)
        row = np.zeros((n + 63) // 64, dtype=np.uint64)
        ns = lib().orc_update_range(self._h, t, n, _ptr(v, C.c_float), _ptr(ref, C.c_int32),
                                    _ptr(inp, C.c_int32), _ptr(row, C.c_uint64))
        return row, ns
