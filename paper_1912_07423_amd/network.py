"""Python front end of the simulator: a thin wrapper over the C ABI (include/snn.h).

Every step of the simulation runs in the HIP kernels of libsnn.so; this module only
marshals arguments.  PyTorch, when present, provides the HIP stream and the device
memory (its caching allocator); it performs no part of the simulation.
"""
import ctypes as C

import numpy as np

from . import _lib as L


def _torch_stream_and_allocator(device):
    try:
        import torch
    except ImportError:
        return None, None, None
    if not torch.cuda.is_available():
        return None, None, None
    stream = torch.cuda.current_stream(device)
    alloc_fn = torch.cuda.caching_allocator_alloc
    delete_fn = torch.cuda.caching_allocator_delete

    def _alloc(nbytes, s, ctx):
        try:
            return alloc_fn(int(nbytes), device, stream)
        except Exception:
            return None

    def _free(ptr, nbytes, s, ctx):
        try:
            delete_fn(ptr)
        except Exception:
            pass  # interpreter shutdown: the process is releasing the device anyway

    keep = (L.ALLOC_FN(_alloc), L.FREE_FN(_free))
    alloc = L.Allocator(keep[0], keep[1], None)
    return stream, alloc, keep


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _structs(spec, **extra):
    """ctypes parameter, population and projection arrays of a workload spec."""
    prm = spec["params"]
    fields = {k: prm[k] for k, _ in L.PARAM_FIELDS
              if k not in ("raster_steps", "window", "delivery", "tiles", "block", "grid",
                           "synapse_weights", "plasticity")}
    base = dict(raster_steps=0, window=0, delivery=0, tiles=0, block=0, grid=0, synapse_weights=0,
                plasticity=0)
    base.update(extra)
    p = L.Params(**fields, **base)
    pops = (L.Population * len(spec["pops"]))(
        *[L.Population(q["size"], q.get("excitatory", 1)) for q in spec["pops"]])
    projs_in = spec.get("projs", [])
    projs = (L.Projection * max(1, len(projs_in)))()
    for k, q in enumerate(projs_in):
        projs[k] = L.Projection(q["from"], q["to"], L.PROJ_KIND[q["kind"]], int(q.get("k", 0)),
                                float(q.get("p", 0.0)), float(q["w_mV"]),
                                int(q.get("plastic", 0)), int(q.get("to_span", 1)))
    return p, pops, projs, len(projs_in)


class Network:
    """A network built and simulated on the GPU from a workload spec (see workloads.py).

    Parameters beyond the spec: raster_steps (raster ring capacity), window (max
    steps per update launch; 0 = the delay), delivery ("auto" | "atomic" | "tiled"),
    tiles (target base tiles of the tiled delivery; 0 = auto), block (its workgroup
    size: 256 | 512 | 1024; 0 = auto), grid (its workgroups; 0 = auto), synapse_weights
    ("auto": one weight per source population where the projections allow it, else
    per synapse; "per_synapse": always a weight per synapse), plasticity ("eager" |
    "lazy": how STDP weights are kept current; identical results), torch_memory
    (allocate through torch's caching allocator and run on torch's current stream).
    """

    def __init__(self, spec, raster_steps=1024, window=0, delivery="auto", tiles=0, block=0,
                 grid=0, synapse_weights="auto", plasticity="eager", torch_memory=True, device=0):
        lib = L.load()
        self._lib = lib
        self._h = None
        p, pops, projs, n_projs = _structs(spec, raster_steps=raster_steps, window=window,
                                           delivery=L.DELIVERY[delivery], tiles=tiles,
                                           block=block, grid=grid,
                                           synapse_weights={"auto": 0, "per_synapse": 1}[synapse_weights],
                                           plasticity=L.PLASTICITY[plasticity])
        self._keep = None
        stream_handle = None
        alloc_ptr = None
        if torch_memory:
            stream, alloc, keep = _torch_stream_and_allocator(device)
            if stream is not None:
                self._keep = keep
                self._alloc = alloc
                alloc_ptr = C.byref(alloc)
                stream_handle = stream.cuda_stream or None
        h = C.c_void_p()
        L.check(lib.snn_build_network(C.byref(p), pops, len(spec["pops"]), projs, n_projs,
                                      alloc_ptr, stream_handle, C.byref(h)))
        self._h = h
        self.spec = spec
        inf = self.info()
        self.n = inf["n"]
        self.words = inf["raster_words"]
        self.plastic = bool(inf["plastic"])

    @classmethod
    def _member(cls, batch, handle, spec):
        """A handle to a network owned by a Batch (no ownership taken)."""
        self = cls.__new__(cls)
        self._lib = batch._lib
        self._h = handle
        self._keep = None
        self._batch = batch        # keeps the batch alive while the handle is used
        self.spec = spec
        inf = self.info()
        self.n = inf["n"]
        self.words = inf["raster_words"]
        self.plastic = bool(inf["plastic"])
        return self

    # -- lifecycle --------------------------------------------------------------------
    def close(self):
        if self._h:
            self._lib.snn_destroy(self._h)   # no-op for a batch member
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- simulation -------------------------------------------------------------------
    def step(self):
        L.check(self._lib.snn_step(self._h))

    def run(self, n_steps):
        L.check(self._lib.snn_run(self._h, int(n_steps)))

    def sync(self):
        L.check(self._lib.snn_sync(self._h))

    # -- readback ---------------------------------------------------------------------
    def info(self):
        i = L.Info()
        L.check(self._lib.snn_get_info(self._h, C.byref(i)))
        d = {k: getattr(i, k) for k, _ in L.Info._fields_ if not k.startswith("pad")}
        d["delivery_name"] = L.DELIVERY_NAME.get(d["delivery"], "?")
        return d

    @property
    def t(self):
        return self.info()["t"]

    @property
    def events(self):
        return self.info()["events"]

    def raster_bits(self, t0, t1):
        out = np.zeros((max(t1 - t0, 0), self.words), dtype=np.uint64)
        L.check(self._lib.snn_get_raster_bits(self._h, t0, t1, _ptr(out)))
        return out

    def raster(self, t0, t1):
        """Boolean spike matrix [t1 - t0, n]."""
        rows = self.raster_bits(t0, t1)
        bits = np.unpackbits(rows.view(np.uint8), axis=1, bitorder="little")
        return bits[:, : self.n].astype(bool)

    def spikes(self, t0, t1):
        """(steps, ids) sorted by step then id."""
        n = C.c_uint64()
        st = self._lib.snn_get_raster(self._h, t0, t1, None, None, 0, C.byref(n))
        if st not in (L.SNN_OK, L.SNN_E_OVERFLOW):
            L.check(st)
        steps = np.zeros(n.value, dtype=np.uint32)
        ids = np.zeros(n.value, dtype=np.uint32)
        L.check(self._lib.snn_get_raster(self._h, t0, t1, _ptr(steps), _ptr(ids), n.value,
                                         C.byref(n)))
        return steps, ids

    def state(self, queues=False, weights=False):
        inf = self.info()
        n, nb, ns = inf["n"], inf["input_buffers"], inf["queue_slots"]
        s = {"v": np.zeros(n, np.float32), "ref": np.zeros(n, np.int32),
             "input": np.zeros((nb, n), np.int32), "x_pre": np.zeros(n, np.float32),
             "x_post": np.zeros(n, np.float32)}
        if queues:
            s["queue"] = np.zeros((ns, inf["queue_stride"]), np.int32)
            s["queue_len"] = np.zeros((ns, inf["queue_groups"]), np.uint32)
        if weights:
            s["w_f32"] = np.zeros(inf["nnz"], np.float32)
        st = L.State(*[_ptr(s.get(k)) for k in ("v", "ref", "input", "x_pre", "x_post", "queue",
                                                 "queue_len", "w_f32")])
        L.check(self._lib.snn_get_state(self._h, C.byref(st)))
        return s

    def set_state(self, **arrays):
        dtypes = {"v": np.float32, "ref": np.int32, "input": np.int32, "x_pre": np.float32,
                  "x_post": np.float32, "queue": np.int32, "queue_len": np.uint32,
                  "w_f32": np.float32}
        conv = {k: np.ascontiguousarray(v, dtype=dtypes[k]) for k, v in arrays.items()}
        st = L.State(*[_ptr(conv.get(k)) for k in ("v", "ref", "input", "x_pre", "x_post", "queue",
                                                    "queue_len", "w_f32")])
        L.check(self._lib.snn_set_state(self._h, C.byref(st)))

    def row(self, i):
        n = C.c_uint64()
        st = self._lib.snn_get_row(self._h, i, None, None, None, 0, C.byref(n))
        if st not in (L.SNN_OK, L.SNN_E_OVERFLOW):
            L.check(st)
        col = np.zeros(n.value, np.int32)
        w = np.zeros(n.value, np.float32 if self.plastic else np.int32)
        wq, wf = (None, w) if self.plastic else (w, None)
        L.check(self._lib.snn_get_row(self._h, i, _ptr(col), _ptr(wq), _ptr(wf), n.value,
                                      C.byref(n)))
        return col, w

    def synapses(self):
        inf = self.info()
        rp = np.zeros(inf["n"] + 1, np.uint64)
        col = np.zeros(inf["nnz"], np.int32)
        w = np.zeros(inf["nnz"], np.float32 if self.plastic else np.int32)
        wq, wf = (None, w) if self.plastic else (w, None)
        L.check(self._lib.snn_get_synapses(self._h, _ptr(rp), _ptr(col), _ptr(wq), _ptr(wf)))
        return rp, col, w

    def drive_table(self):
        t = np.zeros(256, np.uint64)
        L.check(self._lib.snn_get_drive_table(self._h, _ptr(t), 256))
        return t[: self.info()["table_len"]]

    # -- measurement ------------------------------------------------------------------
    def set_profiling(self, on):
        L.check(self._lib.snn_set_profiling(self._h, 1 if on else 0))

    def profile(self):
        p = L.Profile()
        L.check(self._lib.snn_get_profile(self._h, C.byref(p)))
        return {k: getattr(p, k) for k, _ in L.Profile._fields_}

    def reset_profile(self):
        L.check(self._lib.snn_reset_profile(self._h))

    def set_delivery(self, delivery="auto", tiles=0, block=0, grid=0):
        L.check(self._lib.snn_set_delivery(self._h, L.DELIVERY[delivery], tiles, block, grid))

    def autotune_delivery(self, reps=5):
        """Time the delivery configurations on the latest window's spikes; keep the
        fastest (returned as a dict)."""
        t = L.DeliveryTuning()
        L.check(self._lib.snn_autotune_delivery(self._h, reps, C.byref(t)))
        return {"delivery": L.DELIVERY_NAME.get(t.delivery, "?"), "tiles": t.tiles, "block": t.block,
                "grid": t.grid, "ms_per_launch": t.ms_per_launch, "events_per_launch": t.events_per_launch}

    def time_delivery(self, ids, reps=10, steps=0, step_counts=None):
        """Mean time (ms) of one delivery launch over the given spike ids as one window of
        `steps` emission steps (0: the network's window) -- spread evenly, or step w
        taking the next step_counts[w] ids -- and the events per launch."""
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        counts = None if step_counts is None else np.ascontiguousarray(step_counts, dtype=np.uint32)
        if counts is not None and steps == 0:
            steps = len(counts)
        ms = C.c_double()
        ev = C.c_uint64()
        L.check(self._lib.snn_time_delivery(self._h, _ptr(ids), len(ids), _ptr(counts), steps, reps,
                                            C.byref(ms), C.byref(ev)))
        return ms.value, ev.value

    def time_delivery_static(self, ids, reps=10, steps=0, step_counts=None):
        """time_delivery with every device buffer in the library's fixed device array (no
        device allocation; the mean runs over back-to-back launches)."""
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        counts = None if step_counts is None else np.ascontiguousarray(step_counts, dtype=np.uint32)
        if counts is not None and steps == 0:
            steps = len(counts)
        ms = C.c_double()
        ev = C.c_uint64()
        L.check(self._lib.snn_time_delivery_static(self._h, _ptr(ids), len(ids), _ptr(counts), steps, reps,
                                                   C.byref(ms), C.byref(ev)))
        return ms.value, ev.value


class Batch:
    """Many independent static networks stepped together by one persistent launch per
    run (include/snn.h, batched form).  `specs` is a list of workload specs; member k
    is available as a Network handle through `network(k)` for every reader."""

    def __init__(self, specs, raster_steps=1024, torch_memory=True, device=0):
        lib = L.load()
        self._lib = lib
        self._h = None
        self.specs = list(specs)
        keep = []
        members = (L.BatchMember * max(1, len(self.specs)))()
        for k, spec in enumerate(self.specs):
            p, pops, projs, n_projs = _structs(spec)
            keep.append((p, pops, projs))
            members[k] = L.BatchMember(C.pointer(p), pops, projs, len(spec["pops"]), n_projs)
        self._keep = None
        alloc_ptr, stream_handle = None, None
        if torch_memory:
            stream, alloc, kp = _torch_stream_and_allocator(device)
            if stream is not None:
                self._keep = kp
                self._alloc = alloc
                alloc_ptr = C.byref(alloc)
                stream_handle = stream.cuda_stream or None
        h = C.c_void_p()
        L.check(lib.snn_build_batch(members, len(self.specs), raster_steps, alloc_ptr,
                                    stream_handle, C.byref(h)))
        self._h = h
        self._members = {}

    def __len__(self):
        return len(self.specs)

    def close(self):
        if self._h:
            for m in self._members.values():
                m._h = None
            self._members.clear()
            self._lib.snn_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def run(self, n_steps):
        L.check(self._lib.snn_batch_run(self._h, int(n_steps)))

    def sync(self):
        L.check(self._lib.snn_batch_sync(self._h))

    def network(self, k):
        if k not in self._members:
            h = C.c_void_p()
            L.check(self._lib.snn_batch_network(self._h, int(k), C.byref(h)))
            self._members[k] = Network._member(self, h, self.specs[k])
        return self._members[k]

    @staticmethod
    def _tuning_dict(t):
        return {"block": t.block, "per_lane": t.per_lane, "degree_div": t.degree_div,
                "ms_per_step": t.ms_per_step}

    def autotune(self, trial_steps=200):
        t = L.BatchTuning()
        L.check(self._lib.snn_batch_autotune(self._h, int(trial_steps), C.byref(t)))
        return self._tuning_dict(t)

    def tuning(self):
        t = L.BatchTuning()
        L.check(self._lib.snn_batch_get_tuning(self._h, C.byref(t)))
        return self._tuning_dict(t)

    def set_tuning(self, block, degree_div):
        t = L.BatchTuning(block=int(block), degree_div=int(degree_div))
        L.check(self._lib.snn_batch_set_tuning(self._h, C.byref(t)))


def memory_cache_stats(device=0):
    """The library's device-memory cache on `device` (used by objects built with
    torch_memory=False): kept bytes and blocks, and requests served from the cache
    (hits) or by hipMalloc (misses)."""
    lib = L.load()
    vals = [C.c_uint64() for _ in range(4)]
    L.check(lib.snn_memory_cache_stats(device, *[C.byref(v) for v in vals]))
    return dict(zip(("bytes", "blocks", "hits", "misses"), (v.value for v in vals)))


def memory_cache_release(device=-1):
    """Return the cache's kept blocks of `device` (every device if negative) to HIP."""
    L.check(L.load().snn_memory_cache_release(device))
