"""Python binding of libbbc.so (include/bbc.h): argument marshalling only.

Device buffers are torch tensors; every step of the computation runs in the
library's HIP kernels.  There is no fallback: if the library is missing or
the device is not a gfx950 GPU, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbbc.so")

OK, EINVAL, EOFFSETS, ERANGE, ESIGN, EDUP, ENOMEM, EDEVICE, ETOOBIG, EOVERFLOW = range(10)
SIDE_AUTO, SIDE_U, SIDE_V, SIDE_MIN_WEDGES = 0, 1, 2, 3
SCHED_DYNAMIC, SCHED_STATIC = 0, 1
_SCHEDS = {"dynamic": SCHED_DYNAMIC, "static": SCHED_STATIC, SCHED_DYNAMIC: SCHED_DYNAMIC,
           SCHED_STATIC: SCHED_STATIC}
CHECK_SIGNS, CHECK_DUPLICATES, CHECK_ALL = 1, 2, 3
# instantiated wedge-kernel shapes (band_words, wg_size); the first is the default
WEDGE_SHAPES = [(8192, 256), (16384, 512), (16384, 256), (8192, 512), (32768, 1024), (16384, 1024),
                (4096, 128), (8192, 128), (4096, 256)]
_SIDES = {"auto": SIDE_AUTO, "u": SIDE_U, "v": SIDE_V, "min_wedges": SIDE_MIN_WEDGES, SIDE_AUTO: SIDE_AUTO,
          SIDE_U: SIDE_U, SIDE_V: SIDE_V, SIDE_MIN_WEDGES: SIDE_MIN_WEDGES}


class BbcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"bbc status {status}: {message}")
        self.status = status
        self.message = message


class DenseBlock(ctypes.Structure):
    _fields_ = [
        ("n_u_ids", ctypes.c_int32),
        ("n_v_ids", ctypes.c_int32),
        ("u_ids", ctypes.c_void_p),
        ("v_ids", ctypes.c_void_p),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("side", ctypes.c_int32),
        ("checks", ctypes.c_uint32),
        ("timing", ctypes.c_int32),
        ("band_words", ctypes.c_int32),
        ("wg_size", ctypes.c_int32),
        ("wg_per_cu", ctypes.c_int32),
        ("n_blocks", ctypes.c_int32),
        ("blocks", ctypes.POINTER(DenseBlock)),
        ("no_tuning", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("queue_chunk", ctypes.c_int32),
        ("wave_max_work", ctypes.c_int32),
        ("dense_tile", ctypes.c_int32),
        ("scratch_limit", ctypes.c_int64),
    ]


class PlanOptions(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("side", ctypes.c_int32),
        ("min_degree", ctypes.c_int32),
        ("member_frac", ctypes.c_float),
        ("min_density", ctypes.c_float),
        ("min_anchors", ctypes.c_int32),
        ("min_centres", ctypes.c_int32),
        ("max_tries", ctypes.c_int32),
    ]


class GraphDesc(ctypes.Structure):
    _fields_ = [
        ("n_u", ctypes.c_int32),
        ("n_v", ctypes.c_int32),
        ("n_edges", ctypes.c_int64),
        ("off_base", ctypes.c_int64),
        ("edge_base", ctypes.c_int64),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("side", ctypes.c_int32),
        ("n_anchor", ctypes.c_int32),
        ("n_centre", ctypes.c_int32),
        ("n_edges", ctypes.c_int64),
        ("wedges", ctypes.c_uint64),
        ("bands", ctypes.c_uint64),
        ("grid", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("ms_checks", ctypes.c_float),
        ("ms_build", ctypes.c_float),
        ("ms_count", ctypes.c_float),
        ("ms_total", ctypes.c_float),
        ("ms_dense", ctypes.c_float),
        ("n_blocks", ctypes.c_int32),
        ("dense_ops", ctypes.c_uint64),
        ("wedges_all", ctypes.c_uint64),
        ("band_words", ctypes.c_int32),
        ("tuned", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "struct_size"}


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libbbc.so and declares its C signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() or "
                          f"python -m paper_2601_17707_amd.build")
    # torch first: it brings its own HIP runtime, and the library must bind
    # to that same runtime (loaded after it, its libamdhip64 resolves to the
    # copy already in the process) rather than start a second one
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.bbc_options_init.argtypes = [ctypes.POINTER(Options)]
    lib.bbc_options_init.restype = None
    lib.bbc_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    lib.bbc_create.restype = ctypes.c_int
    lib.bbc_destroy.argtypes = [vp]
    lib.bbc_destroy.restype = ctypes.c_int
    lib.bbc_count.argtypes = [vp, i32, i32, i64, vp, vp, vp, ctypes.POINTER(ctypes.c_uint64), vp,
                              ctypes.POINTER(Options), vp]
    lib.bbc_count.restype = ctypes.c_int
    lib.bbc_count_noalloc.argtypes = lib.bbc_count.argtypes
    lib.bbc_count_noalloc.restype = ctypes.c_int
    PD = ctypes.POINTER(GraphDesc)
    lib.bbc_count_batched.argtypes = [vp, i32, PD, vp, vp, vp, vp, ctypes.POINTER(Options), vp]
    lib.bbc_count_batched.restype = ctypes.c_int
    lib.bbc_batch_plan_create.argtypes = [vp, i32, PD, vp, vp, vp, vp, ctypes.POINTER(Options), ctypes.POINTER(vp)]
    lib.bbc_batch_plan_create.restype = ctypes.c_int
    lib.bbc_batch_launch.argtypes = [vp, vp]
    lib.bbc_batch_launch.restype = ctypes.c_int
    lib.bbc_batch_wait.argtypes = [vp, vp]
    lib.bbc_batch_wait.restype = ctypes.c_int
    lib.bbc_batch_plan_destroy.argtypes = [vp]
    lib.bbc_batch_plan_destroy.restype = ctypes.c_int
    lib.bbc_last_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.bbc_last_stats.restype = ctypes.c_int
    lib.bbc_status_string.argtypes = [ctypes.c_int]
    lib.bbc_status_string.restype = ctypes.c_char_p
    lib.bbc_last_error.argtypes = [vp]
    lib.bbc_last_error.restype = ctypes.c_char_p
    lib.bbc_autotune.argtypes = [vp, i32, i32, i64, vp, vp, vp, i32, ctypes.POINTER(Options), vp]
    lib.bbc_autotune.restype = ctypes.c_int
    lib.bbc_autotune_batched.argtypes = [vp, i32, PD, vp, vp, vp, vp, i32, ctypes.POINTER(Options), vp]
    lib.bbc_autotune_batched.restype = ctypes.c_int
    lib.bbc_autotune_blocks.argtypes = [vp, i32, i32, i64, vp, vp, vp, i32, ctypes.POINTER(PlanOptions),
                                        ctypes.POINTER(Options), vp]
    lib.bbc_autotune_blocks.restype = ctypes.c_int
    lib.bbc_tune_save.argtypes = [vp, ctypes.c_char_p]
    lib.bbc_tune_save.restype = ctypes.c_int
    lib.bbc_tune_load.argtypes = [vp, ctypes.c_char_p]
    lib.bbc_tune_load.restype = ctypes.c_int
    lib.bbc_count_classes.argtypes = [vp, i32, i32, i64, vp, vp, vp, ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(Options), vp]
    lib.bbc_count_classes.restype = ctypes.c_int
    lib.bbc_count_classes_per_vertex.argtypes = [vp, i32, i32, i64, vp, vp, vp, ctypes.POINTER(ctypes.c_uint64),
                                                 vp, ctypes.POINTER(Options), vp]
    lib.bbc_count_classes_per_vertex.restype = ctypes.c_int
    lib.bbc_count_bicliques.argtypes = [vp, i32, i32, i64, vp, vp, vp, i32, ctypes.POINTER(ctypes.c_uint64),
                                        ctypes.POINTER(Options), vp]
    lib.bbc_count_bicliques.restype = ctypes.c_int
    lib.bbc_update_delta.argtypes = [vp, i32, i32, i64, vp, vp, vp, i32, vp, vp, vp, ctypes.POINTER(ctypes.c_int64), vp,
                                     vp]
    lib.bbc_update_delta.restype = ctypes.c_int
    lib.bbc_set_update_task_cap.argtypes = [vp, i32]
    lib.bbc_set_update_task_cap.restype = ctypes.c_int
    lib.bbc_plan_options_init.argtypes = [ctypes.POINTER(PlanOptions)]
    lib.bbc_plan_options_init.restype = ctypes.c_int
    lib.bbc_plan_blocks.argtypes = [vp, i32, i32, i64, vp, vp, ctypes.POINTER(PlanOptions), i32,
                                    ctypes.POINTER(DenseBlock), vp, i64, ctypes.POINTER(ctypes.c_int32), vp]
    lib.bbc_plan_blocks.restype = ctypes.c_int
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load_library().bbc_status_string(status).decode()


def options(side="auto", checks=CHECK_ALL, timing=False, band_words=0, wg_size=0, wg_per_cu=0,
            blocks=None, no_tuning=False, schedule="dynamic", queue_chunk=0, wave_max_work=0,
            scratch_limit=0, dense_tile=0) -> Options:
    """Options struct.  ``blocks``: list of (u_ids, v_ids) int32 device
    tensors naming dense blocks (kept alive by the returned object).
    ``schedule``: "dynamic" (shared queue) or "static" (fixed deal).
    ``queue_chunk``: workgroup-regime anchors per queue pop (0 = 1);
    ``wave_max_work``: wave-regime threshold in wedges (0 = the shape's
    largest, -1 = no wave regime); ``scratch_limit``: bytes of scratch the
    call may need (0 = no limit; beyond it the call fails with ENOMEM);
    ``dense_tile``: int8 matrix output tile, 64 or 128 (0 = tuned, else 128)."""
    o = Options()
    load_library().bbc_options_init(ctypes.byref(o))
    o.side = _SIDES[side]
    o.checks = checks
    o.timing = 1 if timing else 0
    o.band_words = band_words
    o.wg_size = wg_size
    o.wg_per_cu = wg_per_cu
    o.no_tuning = 1 if no_tuning else 0
    o.schedule = _SCHEDS[schedule]
    o.queue_chunk = int(queue_chunk)
    o.wave_max_work = int(wave_max_work)
    o.scratch_limit = int(scratch_limit)
    o.dense_tile = int(dense_tile)
    if blocks:
        arr = (DenseBlock * len(blocks))()
        for i, (uids, vids) in enumerate(blocks):
            arr[i].n_u_ids, arr[i].n_v_ids = int(uids.numel()), int(vids.numel())
            arr[i].u_ids, arr[i].v_ids = uids.data_ptr(), vids.data_ptr()
        o.n_blocks = len(blocks)
        o.blocks = ctypes.cast(arr, ctypes.POINTER(DenseBlock))
        o._keep = (arr, blocks)
    return o


def plan_options(side="auto", **kw) -> PlanOptions:
    """Dense-block planner options (defaults from bbc_plan_options_init);
    keyword arguments override fields by name."""
    o = PlanOptions()
    load_library().bbc_plan_options_init(ctypes.byref(o))
    o.side = _SIDES[side]
    for k, v in kw.items():
        if k not in dict(PlanOptions._fields_):
            raise TypeError(f"unknown plan option {k}")
        setattr(o, k, v)
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() > 0 else 0)


def _stream_ptr(stream, like):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream(like.device)
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0))


def _check_tensor(name, t, dtype, torch):
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """One bbc_ctx (scratch arena, events) bound to a device."""

    def __init__(self, device: int | None = None):
        import torch

        self._lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        st = self._lib.bbc_create(self.device, ctypes.byref(h))
        if st != OK:
            raise BbcError(st, f"bbc_create(device={self.device}) failed: {status_string(st)}")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.bbc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def last_error(self) -> str:
        return self._lib.bbc_last_error(self._h).decode()

    def count(self, offsets, adj, signs, n_v: int, per_vertex=None, opts: Options | None = None,
              stream=None) -> int:
        """Balanced butterfly count of the CSR (offsets, adj, signs) over U.

        ``per_vertex``: optional uint64-compatible device tensor (torch.int64)
        of n_u + n_v entries that receives per-vertex counts.
        """
        import torch

        _check_tensor("offsets", offsets, torch.int32, torch)
        _check_tensor("adj", adj, torch.int32, torch)
        _check_tensor("signs", signs, torch.int8, torch)
        n_u = offsets.numel() - 1
        if per_vertex is not None:
            _check_tensor("per_vertex", per_vertex, torch.int64, torch)
            if per_vertex.numel() != n_u + n_v:
                raise ValueError("per_vertex must hold n_u + n_v entries")
        sp = _stream_ptr(stream, offsets)
        out = ctypes.c_uint64(0)
        o = opts if opts is not None else options()
        st = self._lib.bbc_count(self._h, n_u, int(n_v), adj.numel(), _ptr(offsets), _ptr(adj), _ptr(signs), ctypes.byref(out),
                _ptr(per_vertex) if per_vertex is not None else None, ctypes.byref(o), sp)
        if st != OK:
            raise BbcError(st, self.last_error())
        return int(out.value)

    def count_noalloc(self, offsets, adj, signs, n_v: int, per_vertex=None, opts: Options | None = None,
                      stream=None) -> int:
        """As count(), through bbc_count_noalloc: the library allocates nothing
        (its scratch is a fixed per-GPU array; larger graphs raise ETOOBIG)."""
        import torch

        _check_tensor("offsets", offsets, torch.int32, torch)
        _check_tensor("adj", adj, torch.int32, torch)
        _check_tensor("signs", signs, torch.int8, torch)
        n_u = offsets.numel() - 1
        if per_vertex is not None:
            _check_tensor("per_vertex", per_vertex, torch.int64, torch)
            if per_vertex.numel() != n_u + n_v:
                raise ValueError("per_vertex must hold n_u + n_v entries")
        sp = _stream_ptr(stream, offsets)
        out = ctypes.c_uint64(0)
        o = opts if opts is not None else options()
        st = self._lib.bbc_count_noalloc(self._h, n_u, int(n_v), adj.numel(), _ptr(offsets), _ptr(adj), _ptr(signs),
                                         ctypes.byref(out), _ptr(per_vertex) if per_vertex is not None else None,
                                         ctypes.byref(o), sp)
        if st != OK:
            raise BbcError(st, self.last_error())
        return int(out.value)

    def count_classes(self, offsets, adj, signs, n_v: int, opts: Options | None = None, stream=None) -> list:
        """The six sign-pattern classes [++/++, ++/--, --/--, +-/+-, ++/+-,
        +-/--] over pairs of the anchor side (``options(side=...)``)."""
        import torch

        _check_tensor("offsets", offsets, torch.int32, torch)
        _check_tensor("adj", adj, torch.int32, torch)
        _check_tensor("signs", signs, torch.int8, torch)
        out = (ctypes.c_uint64 * 6)()
        o = opts if opts is not None else options()
        st = self._lib.bbc_count_classes(self._h, offsets.numel() - 1, int(n_v), adj.numel(), _ptr(offsets),
                                         _ptr(adj), _ptr(signs), out, ctypes.byref(o), _stream_ptr(stream, offsets))
        if st != OK:
            raise BbcError(st, self.last_error())
        return [int(x) for x in out]

    def count_classes_per_vertex(self, offsets, adj, signs, n_v: int, per_vertex, opts: Options | None = None,
                                 stream=None) -> list:
        """The six classes in total (returned) and per vertex: per_vertex is a
        device int64 tensor of shape (n_u + n_v, 6), U first, overwritten."""
        import torch

        _check_tensor("offsets", offsets, torch.int32, torch)
        _check_tensor("adj", adj, torch.int32, torch)
        _check_tensor("signs", signs, torch.int8, torch)
        _check_tensor("per_vertex", per_vertex, torch.int64, torch)
        n_u = offsets.numel() - 1
        if per_vertex.numel() != (n_u + int(n_v)) * 6:
            raise ValueError("per_vertex must hold (n_u + n_v) x 6 entries")
        out = (ctypes.c_uint64 * 6)()
        o = opts if opts is not None else options()
        st = self._lib.bbc_count_classes_per_vertex(self._h, n_u, int(n_v), adj.numel(), _ptr(offsets), _ptr(adj),
                                                    _ptr(signs), out, _ptr(per_vertex), ctypes.byref(o),
                                                    _stream_ptr(stream, offsets))
        if st != OK:
            raise BbcError(st, self.last_error())
        return [int(x) for x in out]

    def count_bicliques(self, offsets, adj, signs, n_v: int, k: int, opts: Options | None = None,
                        stream=None) -> int:
        """Balanced (2,k)-bicliques with the pair on ``options(side=...)``,
        exact (128-bit) as a Python int."""
        import torch

        _check_tensor("offsets", offsets, torch.int32, torch)
        _check_tensor("adj", adj, torch.int32, torch)
        _check_tensor("signs", signs, torch.int8, torch)
        out = (ctypes.c_uint64 * 2)()
        o = opts if opts is not None else options()
        st = self._lib.bbc_count_bicliques(self._h, offsets.numel() - 1, int(n_v), adj.numel(), _ptr(offsets),
                                           _ptr(adj), _ptr(signs), int(k), out, ctypes.byref(o),
                                           _stream_ptr(stream, offsets))
        if st != OK:
            raise BbcError(st, self.last_error())
        return int(out[0]) | (int(out[1]) << 64)

    def update_delta(self, offsets, adj, signs, n_v: int, upd_u, upd_v, upd_state, per_update=None,
                     stream=None) -> int:
        """T(after) - T(before) for a batch of edge updates: pair (upd_u[i],
        upd_v[i]) takes state upd_state[i] (+1 / -1, or 0 = absent).
        ``per_update`` (int64 device tensor, optional) receives each
        update's share."""
        import torch

        _check_tensor("offsets", offsets, torch.int32, torch)
        _check_tensor("adj", adj, torch.int32, torch)
        _check_tensor("signs", signs, torch.int8, torch)
        _check_tensor("upd_u", upd_u, torch.int32, torch)
        _check_tensor("upd_v", upd_v, torch.int32, torch)
        _check_tensor("upd_state", upd_state, torch.int8, torch)
        q = upd_u.numel()
        if upd_v.numel() != q or upd_state.numel() != q:
            raise ValueError("update arrays differ in length")
        if per_update is not None:
            _check_tensor("per_update", per_update, torch.int64, torch)
            if per_update.numel() < q:
                raise ValueError("per_update holds fewer entries than updates")
        out = ctypes.c_int64(0)
        st = self._lib.bbc_update_delta(self._h, offsets.numel() - 1, int(n_v), adj.numel(), _ptr(offsets),
                                        _ptr(adj), _ptr(signs), q, _ptr(upd_u), _ptr(upd_v), _ptr(upd_state),
                                        ctypes.byref(out), _ptr(per_update) if per_update is not None else None,
                                        _stream_ptr(stream, offsets))
        if st != OK:
            raise BbcError(st, self.last_error())
        return int(out.value)

    def set_update_task_cap(self, cap: int) -> None:
        """Tasks per update of update_delta (0 = the default, 4,096)."""
        st = self._lib.bbc_set_update_task_cap(self._h, int(cap))
        if st != OK:
            raise BbcError(st, self.last_error())

    def count_batched(self, batch: "Batch", opts: Options | None = None, stream=None):
        """Per-graph counts of a Batch; returns its totals tensor (int64, on device)."""
        o = opts if opts is not None else options()
        st = self._lib.bbc_count_batched(self._h, batch.n_graphs, batch.descs, _ptr(batch.offsets),
                                         _ptr(batch.adj), _ptr(batch.signs), _ptr(batch.totals),
                                         ctypes.byref(o), _stream_ptr(stream, batch.offsets))
        if st != OK:
            raise BbcError(st, self.last_error())
        return batch.totals

    @staticmethod
    def _chosen(o) -> dict:
        return dict(band_words=o.band_words, wg_size=o.wg_size, wg_per_cu=o.wg_per_cu, schedule=o.schedule,
                    queue_chunk=o.queue_chunk, wave_max_work=o.wave_max_work)

    def autotune(self, offsets, adj, signs, n_v: int, reps: int = 2, stream=None) -> dict:
        """Times the wedge kernel's shapes, grids, schedules, queue chunks and
        wave-regime thresholds on this calibration graph and records the
        fastest for its size class; returns the choice."""
        import torch

        _check_tensor("offsets", offsets, torch.int32, torch)
        _check_tensor("adj", adj, torch.int32, torch)
        _check_tensor("signs", signs, torch.int8, torch)
        chosen = Options()
        st = self._lib.bbc_autotune(self._h, offsets.numel() - 1, int(n_v), adj.numel(), _ptr(offsets), _ptr(adj),
                                    _ptr(signs), int(reps), ctypes.byref(chosen), _stream_ptr(stream, offsets))
        if st != OK:
            raise BbcError(st, self.last_error())
        return self._chosen(chosen)

    def autotune_batched(self, batch: "Batch", reps: int = 2, stream=None) -> dict:
        """The same search on a batch, recorded under the batch's size class
        (used by count_batched and plans of that layout)."""
        chosen = Options()
        st = self._lib.bbc_autotune_batched(self._h, batch.n_graphs, batch.descs, _ptr(batch.offsets),
                                            _ptr(batch.adj), _ptr(batch.signs), _ptr(batch.totals), int(reps),
                                            ctypes.byref(chosen), _stream_ptr(stream, batch.offsets))
        if st != OK:
            raise BbcError(st, self.last_error())
        return self._chosen(chosen)

    def autotune_blocks(self, offsets, adj, signs, n_v: int, reps: int = 2, stream=None) -> dict:
        """Times the planner's degree threshold and the int8 tile on this
        graph (every hybrid count checked against the sparse-only one) and
        records the fastest for its size class."""
        import torch

        _check_tensor("offsets", offsets, torch.int32, torch)
        _check_tensor("adj", adj, torch.int32, torch)
        _check_tensor("signs", signs, torch.int8, torch)
        cp, co = PlanOptions(), Options()
        st = self._lib.bbc_autotune_blocks(self._h, offsets.numel() - 1, int(n_v), adj.numel(), _ptr(offsets),
                                           _ptr(adj), _ptr(signs), int(reps), ctypes.byref(cp), ctypes.byref(co),
                                           _stream_ptr(stream, offsets))
        if st != OK:
            raise BbcError(st, self.last_error())
        return dict(min_degree=cp.min_degree, dense_tile=co.dense_tile)

    def tune_save(self, path: str):
        st = self._lib.bbc_tune_save(self._h, os.fsencode(path))
        if st != OK:
            raise BbcError(st, self.last_error())

    def tune_load(self, path: str):
        st = self._lib.bbc_tune_load(self._h, os.fsencode(path))
        if st != OK:
            raise BbcError(st, self.last_error())

    def plan_blocks(self, offsets, adj, n_v: int, opts: PlanOptions | None = None, max_blocks: int = 64,
                    stream=None) -> list:
        """Dense blocks found by the planner, as (u_ids, v_ids) int32 device
        tensors ready for ``options(blocks=...)``."""
        import torch

        _check_tensor("offsets", offsets, torch.int32, torch)
        _check_tensor("adj", adj, torch.int32, torch)
        n_u = offsets.numel() - 1
        o = opts if opts is not None else plan_options()
        cap = min(n_u + int(n_v), max_blocks * (16384 + 65535))
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device=offsets.device)
        arr = (DenseBlock * max(max_blocks, 1))()
        nb = ctypes.c_int32(0)
        st = self._lib.bbc_plan_blocks(self._h, n_u, int(n_v), adj.numel(), _ptr(offsets), _ptr(adj),
                                       ctypes.byref(o), int(max_blocks), arr, ctypes.c_void_p(ids.data_ptr()),
                                       cap, ctypes.byref(nb), _stream_ptr(stream, offsets))
        if st != OK:
            raise BbcError(st, self.last_error())
        out, base = [], ids.data_ptr()
        for i in range(nb.value):
            b = arr[i]
            pu, pv = (b.u_ids - base) // 4, (b.v_ids - base) // 4
            out.append((ids[pu:pu + b.n_u_ids], ids[pv:pv + b.n_v_ids]))
        return out

    def plan(self, batch: "Batch", opts: Options | None = None) -> "BatchPlan":
        return BatchPlan(self, batch, opts)

    def stats(self) -> dict:
        s = Stats()
        s.struct_size = ctypes.sizeof(Stats)
        self._lib.bbc_last_stats(self._h, ctypes.byref(s))
        return s.as_dict()


_default = {}


def default_context(device: int | None = None) -> Context:
    import torch

    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _default:
        _default[dev] = Context(dev)
    return _default[dev]


def graph_tensors(g, device="cuda"):
    """(offsets, adj, signs) device tensors of a CSR graph object."""
    import numpy as np
    import torch

    off = torch.from_numpy(np.ascontiguousarray(g.offsets, np.int32)).to(device)
    adj = torch.from_numpy(np.ascontiguousarray(g.adj, np.int32)).to(device)
    sg = torch.from_numpy(np.ascontiguousarray(g.signs, np.int8)).to(device)
    return off, adj, sg


def count(g, per_vertex: bool = False, side="auto", checks=CHECK_ALL, blocks=None, ctx: Context | None = None,
          **kw):
    """Counts a graph object (n_u, n_v, offsets, adj, signs) on the current GPU.

    ``blocks``: optional list of (u_ids, v_ids) integer arrays naming dense
    blocks.  Returns the total, or (total, per-vertex int64 tensor) with
    per_vertex.
    """
    import torch

    ctx = ctx or default_context()
    dev = f"cuda:{ctx.device}"
    off, adj, sg = graph_tensors(g, dev)
    pv = torch.empty(int(g.n_u) + int(g.n_v), dtype=torch.int64, device=off.device) if per_vertex else None
    dblocks = None
    if blocks is not None:
        dblocks = [(torch.as_tensor(np.asarray(u, np.int32)).to(dev), torch.as_tensor(np.asarray(v, np.int32)).to(dev))
                   for u, v in blocks]
    t = ctx.count(off, adj, sg, int(g.n_v), per_vertex=pv,
                  opts=options(side=side, checks=checks, blocks=dblocks, **kw))
    return (t, pv) if per_vertex else t


class Batch:
    """Device-resident batch of graphs: concatenated CSR arrays, descriptors
    and a totals tensor (int64, one per graph)."""

    def __init__(self, graphs, device="cuda", layout=None):
        """``layout`` (optional) lists, per graph, (off_base, edge_base) to
        place graphs anywhere in larger arrays; by default graphs are packed
        end to end."""
        import numpy as np
        import torch

        n = len(graphs)
        self.n_graphs = n
        descs = (GraphDesc * max(n, 1))()
        if layout is None:
            ob, eb = 0, 0
            layout = []
            for g in graphs:
                layout.append((ob, eb))
                ob += int(g.n_u) + 1
                eb += int(g.m)
        n_off = max([ob + int(g.n_u) + 1 for (ob, _), g in zip(layout, graphs)] + [1])
        n_edge = max([eb + int(g.m) for (_, eb), g in zip(layout, graphs)] + [1])
        off = np.zeros(n_off, np.int32)
        adj = np.zeros(n_edge, np.int32)
        sg = np.ones(n_edge, np.int8)
        for i, (g, (ob, eb)) in enumerate(zip(graphs, layout)):
            off[ob: ob + g.n_u + 1] = g.offsets
            adj[eb: eb + g.m] = g.adj
            sg[eb: eb + g.m] = g.signs
            descs[i].n_u, descs[i].n_v, descs[i].n_edges = int(g.n_u), int(g.n_v), int(g.m)
            descs[i].off_base, descs[i].edge_base = int(ob), int(eb)
        self.descs = descs
        self.offsets = torch.from_numpy(off).to(device)
        self.adj = torch.from_numpy(adj).to(device)
        self.signs = torch.from_numpy(sg).to(device)
        self.totals = torch.zeros(max(n, 1), dtype=torch.int64, device=device)


class BatchPlan:
    """A captured batch pipeline (bbc_batch_plan): launch() replays it."""

    def __init__(self, ctx: Context, batch: Batch, opts: Options | None = None):
        self._lib = ctx._lib
        self.ctx = ctx
        self.batch = batch  # keeps the captured buffers alive
        o = opts if opts is not None else options()
        h = ctypes.c_void_p()
        st = self._lib.bbc_batch_plan_create(ctx._h, batch.n_graphs, batch.descs, _ptr(batch.offsets),
                                             _ptr(batch.adj), _ptr(batch.signs), _ptr(batch.totals),
                                             ctypes.byref(o), ctypes.byref(h))
        if st != OK:
            raise BbcError(st, ctx.last_error())
        self._h = h

    def launch(self, stream=None):
        st = self._lib.bbc_batch_launch(self._h, _stream_ptr(stream, self.batch.offsets))
        if st != OK:
            raise BbcError(st, self.ctx.last_error())

    def wait(self, stream=None):
        st = self._lib.bbc_batch_wait(self._h, _stream_ptr(stream, self.batch.offsets))
        if st != OK:
            raise BbcError(st, self.ctx.last_error())
        return self.batch.totals

    def close(self):
        if getattr(self, "_h", None):
            self._lib.bbc_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
