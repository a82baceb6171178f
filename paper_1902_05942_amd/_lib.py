"""ctypes binding of libpf.so (include/pf.h): argument marshalling only.

Every function here has the name of the C entry point without the pf_
prefix, takes torch tensors where the C function takes device pointers, and
enqueues on torch's current HIP stream unless a stream is given.  No step of
the filter runs in Python or in PyTorch; if the library is missing the
import fails.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpf.so")

PF_OK, PF_EINVAL, PF_ERANGE, PF_ELAUNCH = 0, -1, -2, -3
V_INVALID, V_KEYRANGE, V_OVERFLOW, V_RADRANGE = 1, 2, 4, 8
STAT_USED, STAT_DISP, STAT_OVERFLOW, STAT_TEMPORAL_HIT, STAT_HIST, STATS_LEN = 0, 1, 2, 3, 8, 128
SUMS_FIXED64, SUMS_FLOAT32 = 0, 1
CELL_BYTES = 32
SLOT_BYTES = 64  # a slot record: cell at 0, key at 32, temporal value at 48


class PfError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__(f"{fn} returned {status}")
        self.status = status


class pf_table(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_void_p), ("key", ctypes.c_void_p), ("blend", ctypes.c_void_p),
                ("occ", ctypes.c_void_p), ("stats", ctypes.c_void_p), ("log2_slots", ctypes.c_uint32),
                ("max_probe", ctypes.c_uint32), ("frac_bits", ctypes.c_int32), ("sum_format", ctypes.c_uint32)]


class pf_history(ctypes.Structure):
    _fields_ = [("slot", ctypes.c_void_p), ("stamp", ctypes.c_void_p), ("log2_slots", ctypes.c_uint32),
                ("max_age", ctypes.c_uint32)]


class pf_key_params(ctypes.Structure):
    _fields_ = [("cam", ctypes.c_float * 3), ("s", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("idx_base", ctypes.c_uint64)]


class pf_mlp(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("wb", ctypes.c_void_p), ("m", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("partial", ctypes.c_void_p), ("loss", ctypes.c_void_p), ("max_batch", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class pf_geometry(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("px", ctypes.c_void_p), ("py", ctypes.c_void_p), ("pz", ctypes.c_void_p),
                ("nx", ctypes.c_void_p), ("ny", ctypes.c_void_p), ("nz", ctypes.c_void_p),
                ("cam", ctypes.c_float * 3), ("reserved", ctypes.c_float)]


MLP_NPARAM, MLP_IN, MLP_BLOCK_SAMPLES = 10384, 80, 64


class pf_view(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("px", "py", "pz", "nx", "ny", "nz", "valid", "r", "g", "b", "key",
                                                "vflags", "slot", "r_out", "g_out", "b_out", "count_out")] + [
        ("cur", pf_table), ("prev", pf_table), ("kp", pf_key_params), ("n", ctypes.c_uint32),
        ("alpha_old", ctypes.c_float), ("temporal", ctypes.c_int32), ("reserved", ctypes.c_uint32)]


MAX_VIEWS = 64


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() or "
                          "python paper_1902_05942_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32, f32, i = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32,
                                 ctypes.c_float, ctypes.c_int)
    T = ctypes.POINTER(pf_table)
    sig = {
        "pf_version": ([], ctypes.c_char_p),
        "pf_table_bytes": ([u32, i], ctypes.c_size_t),
        "pf_table_carve": ([vp, u32, i, u32, i32, T], i),
        "pf_table_init": ([T, vp], i),
        "pf_clear": ([T, vp], i),
        "pf_build_keys": ([vp] * 7 + [u64, ctypes.POINTER(pf_key_params), u32, vp, vp, vp, vp, vp], i),
        "pf_insert_accumulate": ([T, vp, vp, vp, vp, vp, vp, u64, u32, vp], i),
        "pf_insert_workspace_bytes": ([u64, u32], ctypes.c_size_t),
        "pf_insert_accumulate_binned": ([T, vp, vp, vp, vp, vp, vp, u64, vp, ctypes.c_size_t, vp], i),
        "pf_build_keys_insert_binned": ([T] + [vp] * 7 + [ctypes.POINTER(pf_key_params), vp, vp, vp, u64, vp, vp, vp,
                                                          vp, ctypes.c_size_t, vp], i),
        "pf_build_keys_insert_binned_noalloc": ([T] + [vp] * 7 + [ctypes.POINTER(pf_key_params), vp, vp, vp, u64, vp,
                                                                  vp, vp, vp], i),
        "pf_query_average": ([T, vp, vp, vp, vp, vp, vp, u64, i, vp, vp, vp, vp, vp], i),
        "pf_query_average_clear": ([T, vp, vp, vp, vp, vp, vp, u64, i, vp, vp, vp, vp, T, vp], i),
        "pf_build_keys_insert_binned_temporal": ([T] + [vp] * 7 + [ctypes.POINTER(pf_key_params), vp, vp, vp, u64, vp,
                                                                   vp, vp, vp, ctypes.c_size_t, T, f32, u32, vp], i),
        "pf_temporal_update": ([T, T, f32, i, vp], i),
        "pf_temporal_integrate": ([T, T, u32, vp], i),
        "pf_low_density_fallback": ([T, u32, i, vp], i),
        "pf_coarsen_keys": ([vp, vp, u64, u32, vp, vp, vp], i),
        "pf_resolve_pixels": ([vp, vp, vp, vp, vp, vp, vp, u64, u32, i, vp, vp, vp, vp], i),
        "pf_history_bytes": ([u32], ctypes.c_size_t),
        "pf_history_carve": ([vp, u32, u32, ctypes.POINTER(pf_history)], i),
        "pf_history_init": ([ctypes.POINTER(pf_history), vp], i),
        "pf_temporal_history": ([T, ctypes.POINTER(pf_history), f32, i, u32, u32, vp], i),
        "pf_query_multilevel": ([T, T, vp, vp, vp, vp, vp, vp, vp, u64, u32, i, vp, vp, vp, vp, vp], i),
        "pf_read_stats": ([T, vp, vp], i),
        "pf_views_workspace_bytes": ([ctypes.POINTER(u64), ctypes.POINTER(u32), u32], ctypes.c_size_t),
        "pf_filter_views": ([ctypes.POINTER(pf_view), u32, u32, u32, u32, vp, ctypes.c_size_t, vp], i),
        "pf_views_concurrent_workspace_bytes": ([ctypes.POINTER(u64), ctypes.POINTER(u32), u32], ctypes.c_size_t),
        "pf_filter_views_concurrent": ([ctypes.POINTER(pf_view), u32, u32, vp, ctypes.c_size_t, vp], i),
        "pf_mlp_bytes": ([u32], ctypes.c_size_t),
        "pf_mlp_carve": ([vp, u32, ctypes.POINTER(pf_mlp)], i),
        "pf_mlp_init": ([ctypes.POINTER(pf_mlp), vp], i),
        "pf_mlp_select_workspace_bytes": ([u64], ctypes.c_size_t),
        "pf_mlp_select": ([vp, vp, u64, u32, u32, vp, vp, vp, vp, vp], i),
        "pf_mlp_train_step": ([ctypes.POINTER(pf_mlp), T, ctypes.POINTER(pf_geometry), vp, vp, vp, u32, u64, u32, f32,
                               vp], i),
        "pf_mlp_features": ([ctypes.POINTER(pf_geometry), vp, u64, vp, vp], i),
        "pf_mlp_infer": ([ctypes.POINTER(pf_mlp), ctypes.POINTER(pf_geometry), vp, vp, u64, vp, vp, vp, vp], i),
        "pf_microbench": ([i, vp, u64, u32, u32, u64, vp, vp], i),
        "pf_wall_clock_hz": ([], u64),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()

EXPORTED = ("pf_version", "pf_table_bytes", "pf_table_carve", "pf_table_init", "pf_clear", "pf_build_keys",
            "pf_insert_accumulate", "pf_query_average", "pf_temporal_update", "pf_read_stats", "pf_mlp_bytes",
            "pf_mlp_carve", "pf_mlp_init", "pf_mlp_select_workspace_bytes", "pf_mlp_select", "pf_mlp_train_step",
            "pf_mlp_features", "pf_mlp_infer", "pf_views_workspace_bytes", "pf_filter_views",
            "pf_views_concurrent_workspace_bytes", "pf_filter_views_concurrent",
            "pf_insert_workspace_bytes", "pf_insert_accumulate_binned", "pf_microbench",
            "pf_temporal_integrate", "pf_build_keys_insert_binned", "pf_wall_clock_hz", "pf_low_density_fallback",
            "pf_coarsen_keys", "pf_query_multilevel", "pf_history_bytes", "pf_history_carve", "pf_history_init",
            "pf_temporal_history", "pf_resolve_pixels", "pf_query_average_clear",
            "pf_build_keys_insert_binned_temporal", "pf_build_keys_insert_binned_noalloc")


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda, "device tensor expected"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(fn, st):
    if st != PF_OK:
        raise PfError(fn, st)


def version() -> str:
    return lib.pf_version().decode()


def table_bytes(log2_slots: int, with_blend: bool = True) -> int:
    return int(lib.pf_table_bytes(log2_slots, int(with_blend)))


class Table:
    """One table arena (a torch uint8 tensor) carved into the pf_table views."""

    def __init__(self, log2_slots: int, max_probe: int = 64, frac_bits: int = 24, with_blend: bool = True,
                 device="cuda", arena=None, sum_format: int = 0):
        nbytes = table_bytes(log2_slots, with_blend)
        if nbytes == 0:
            raise PfError("pf_table_bytes", PF_ERANGE)
        self.arena = arena if arena is not None else torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.t = pf_table()
        _check("pf_table_carve", lib.pf_table_carve(_ptr(self.arena), log2_slots, int(with_blend), max_probe,
                                                    frac_bits, ctypes.byref(self.t)))
        self.t.sum_format = sum_format
        self.log2_slots = log2_slots
        self.with_blend = with_blend

    @property
    def ref(self):
        return ctypes.byref(self.t)

    def _view(self, addr, nbytes, dtype):
        base = self.arena.data_ptr()
        off = addr - base
        return self.arena[off:off + nbytes].view(dtype)

    def _records(self, dtype, per):
        S = 1 << self.log2_slots
        return self._view(self.t.cell, S * SLOT_BYTES, dtype).view(S, per)

    def cells(self) -> torch.Tensor:
        """[2^m, 8] int32 view: fp, count, sum0 lo/hi, sum1 lo/hi, sum2 lo/hi."""
        return self._records(torch.int32, SLOT_BYTES // 4)[:, :CELL_BYTES // 4]

    def keys(self) -> torch.Tensor:
        return self._records(torch.int64, SLOT_BYTES // 8)[:, 4]

    def blend(self) -> torch.Tensor:
        return self._records(torch.float32, SLOT_BYTES // 4)[:, 12:16]

    def occupancy(self) -> torch.Tensor:
        """Occupancy bitmap as int32 words (bit s % 32 of word s // 32)."""
        S = 1 << self.log2_slots
        return self._view(self.t.occ, (S + 31) // 32 * 4, torch.int32)


def table_init(t: Table, stream=None):
    _check("pf_table_init", lib.pf_table_init(t.ref, _stream(stream)))


def clear(t: Table, stream=None):
    _check("pf_clear", lib.pf_clear(t.ref, _stream(stream)))


def build_keys(px, py, pz, nx, ny, nz, valid, cam, s, seed, idx_base, log2_slots, key, fp, home, vflags,
               stream=None):
    kp = pf_key_params()
    for c in range(3):
        kp.cam[c] = float(cam[c])
    kp.s = float(s)
    kp.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    kp.idx_base = int(idx_base)
    n = key.numel()
    _check("pf_build_keys", lib.pf_build_keys(_ptr(px), _ptr(py), _ptr(pz), _ptr(nx), _ptr(ny), _ptr(nz),
                                              _ptr(valid), n, ctypes.byref(kp), log2_slots, _ptr(key), _ptr(fp),
                                              _ptr(home), _ptr(vflags), _stream(stream)))


def insert_accumulate(t: Table, key, r, g, b, vflags, slot_out=None, agg_width=0, stream=None):
    _check("pf_insert_accumulate", lib.pf_insert_accumulate(t.ref, _ptr(key), _ptr(r), _ptr(g), _ptr(b),
                                                            _ptr(vflags), _ptr(slot_out), key.numel(), agg_width,
                                                            _stream(stream)))


def insert_workspace_bytes(n: int, log2_slots: int) -> int:
    return int(lib.pf_insert_workspace_bytes(n, log2_slots))


def insert_accumulate_binned(t: Table, key, r, g, b, vflags, slot_out, workspace, stream=None):
    _check("pf_insert_accumulate_binned", lib.pf_insert_accumulate_binned(
        t.ref, _ptr(key), _ptr(r), _ptr(g), _ptr(b), _ptr(vflags), _ptr(slot_out), key.numel(), _ptr(workspace),
        workspace.numel() * workspace.element_size(), _stream(stream)))


def build_keys_insert_binned(t: Table, px, py, pz, nx, ny, nz, valid, cam, s, seed, idx_base, r, g, b, key, vflags,
                             slot_out, workspace, stream=None):
    kp = pf_key_params()
    for c in range(3):
        kp.cam[c] = float(cam[c])
    kp.s = float(s)
    kp.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    kp.idx_base = int(idx_base)
    _check("pf_build_keys_insert_binned", lib.pf_build_keys_insert_binned(
        t.ref, _ptr(px), _ptr(py), _ptr(pz), _ptr(nx), _ptr(ny), _ptr(nz), _ptr(valid), ctypes.byref(kp), _ptr(r),
        _ptr(g), _ptr(b), vflags.numel(), _ptr(key), _ptr(vflags), _ptr(slot_out), _ptr(workspace),
        workspace.numel() * workspace.element_size(), _stream(stream)))


NOALLOC_SCRATCH_BYTES, NOALLOC_BATCH = 80 << 20, 1 << 20


def build_keys_insert_binned_noalloc(t: Table, px, py, pz, nx, ny, nz, valid, cam, s, seed, idx_base, r, g, b, key,
                                     vflags, slot_out, stream=None):
    """build_keys_insert_binned without a workspace argument: the library's
    own device scratch (shared by every call on the device) serves as it."""
    kp = pf_key_params()
    for c in range(3):
        kp.cam[c] = float(cam[c])
    kp.s = float(s)
    kp.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    kp.idx_base = int(idx_base)
    _check("pf_build_keys_insert_binned_noalloc", lib.pf_build_keys_insert_binned_noalloc(
        t.ref, _ptr(px), _ptr(py), _ptr(pz), _ptr(nx), _ptr(ny), _ptr(nz), _ptr(valid), ctypes.byref(kp), _ptr(r),
        _ptr(g), _ptr(b), vflags.numel(), _ptr(key), _ptr(vflags), _ptr(slot_out), _stream(stream)))


def build_keys_insert_binned_temporal(t: Table, px, py, pz, nx, ny, nz, valid, cam, s, seed, idx_base, r, g, b, key,
                                      vflags, slot_out, workspace, prev, alpha_old: float = 0.2,
                                      max_samples: int = 0, stream=None):
    """build_keys_insert_binned and the frame's temporal pass (moving
    average with alpha_old, or integration when max_samples > 0) in the same
    launches; t must be empty before the call."""
    kp = pf_key_params()
    for c in range(3):
        kp.cam[c] = float(cam[c])
    kp.s = float(s)
    kp.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    kp.idx_base = int(idx_base)
    _check("pf_build_keys_insert_binned_temporal", lib.pf_build_keys_insert_binned_temporal(
        t.ref, _ptr(px), _ptr(py), _ptr(pz), _ptr(nx), _ptr(ny), _ptr(nz), _ptr(valid), ctypes.byref(kp), _ptr(r),
        _ptr(g), _ptr(b), vflags.numel(), _ptr(key), _ptr(vflags), _ptr(slot_out), _ptr(workspace),
        workspace.numel() * workspace.element_size(), None if prev is None else prev.ref, float(alpha_old),
        int(max_samples), _stream(stream)))


def query_average(t: Table, key, slot, r_in, g_in, b_in, vflags, use_blend, r_out, g_out, b_out, count_out=None,
                  stream=None):
    n = vflags.numel()
    _check("pf_query_average", lib.pf_query_average(t.ref, _ptr(key), _ptr(slot), _ptr(r_in), _ptr(g_in),
                                                    _ptr(b_in), _ptr(vflags), n, int(bool(use_blend)), _ptr(r_out),
                                                    _ptr(g_out), _ptr(b_out), _ptr(count_out), _stream(stream)))


def query_average_clear(t: Table, key, slot, r_in, g_in, b_in, vflags, use_blend, r_out, g_out, b_out,
                        clear: Table, count_out=None, stream=None):
    """query_average on t and clear() of another table in one launch."""
    n = vflags.numel()
    _check("pf_query_average_clear", lib.pf_query_average_clear(
        t.ref, _ptr(key), _ptr(slot), _ptr(r_in), _ptr(g_in), _ptr(b_in), _ptr(vflags), n, int(bool(use_blend)),
        _ptr(r_out), _ptr(g_out), _ptr(b_out), _ptr(count_out), clear.ref, _stream(stream)))


def temporal_update(cur: Table, prev, alpha_old: float, mode: int = 0, stream=None):
    _check("pf_temporal_update", lib.pf_temporal_update(cur.ref, None if prev is None else prev.ref,
                                                        float(alpha_old), mode, _stream(stream)))


MAX_SAMPLES = 1 << 24


def temporal_integrate(cur: Table, prev, max_samples: int = MAX_SAMPLES, stream=None):
    _check("pf_temporal_integrate", lib.pf_temporal_integrate(cur.ref, None if prev is None else prev.ref,
                                                              int(max_samples), _stream(stream)))


LD_NEIGHBOURS, LD_NORMALS = 0, 1
TEMPORAL_ACROSS_LEVELS = 16  # pf_temporal_update mode bit: resolution changes across frames


def low_density_fallback(t: Table, below: int, mode: int = LD_NEIGHBOURS, stream=None):
    """Section 3.3's fallback for cells with fewer than `below` vertices
    (after temporal_update / temporal_integrate, before query_average with
    use_blend)."""
    _check("pf_low_density_fallback", lib.pf_low_density_fallback(t.ref, int(below), int(mode), _stream(stream)))


class History:
    """Voxel values kept across frames with eviction by priority: one arena
    (a torch uint8 tensor) carved into the pf_history arrays, emptied."""

    def __init__(self, log2_slots: int, max_age: int, device="cuda", stream=None):
        nbytes = lib.pf_history_bytes(log2_slots)
        if nbytes == 0:
            raise PfError("pf_history_bytes", PF_ERANGE)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.h = pf_history()
        _check("pf_history_carve", lib.pf_history_carve(_ptr(self.arena), log2_slots, max_age, ctypes.byref(self.h)))
        self.log2_slots, self.max_age = log2_slots, max_age
        _check("pf_history_init", lib.pf_history_init(ctypes.byref(self.h), _stream(stream)))

    @property
    def ref(self):
        return ctypes.byref(self.h)

    def _view(self, addr, nbytes, dtype):
        off = addr - self.arena.data_ptr()
        return self.arena[off:off + nbytes].view(dtype)

    def arrays(self):
        """(word int64, key int64, value float32 [S,4], stamp int32) views of
        the 32-byte slot records and the stamps."""
        S = 1 << self.log2_slots
        rec = self._view(self.h.slot, 32 * S, torch.int64).view(S, 4)
        return (rec[:, 0], rec[:, 1], rec[:, 2:].contiguous().view(torch.float32).view(S, 4),
                self._view(self.h.stamp, 4 * S, torch.int32))


def temporal_history(cur: Table, hist: History, alpha_old: float, mode: int, max_samples: int, frame: int,
                     stream=None):
    _check("pf_temporal_history", lib.pf_temporal_history(cur.ref, hist.ref, float(alpha_old), int(mode),
                                                          int(max_samples), int(frame), _stream(stream)))


def resolve_pixels(r, g, b, throughput, valid, pixels: int, verts_per_path: int, out, accumulate=False, stream=None):
    """Section 3's resolve: out (pr, pg, pb) [pixels] = (out +) sum over each
    pixel's vertices of throughput * value; throughput (tr, tg, tb) or None."""
    tr, tg, tb = throughput if throughput is not None else (None, None, None)
    _check("pf_resolve_pixels", lib.pf_resolve_pixels(_ptr(r), _ptr(g), _ptr(b), _ptr(tr), _ptr(tg), _ptr(tb),
                                                      _ptr(valid), int(pixels), int(verts_per_path), int(accumulate),
                                                      _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _stream(stream)))


def coarsen_keys(key, vflags, levels: int, key_out, vflags_out, stream=None):
    """Keys of the voxels `levels` levels coarser (multi-level accumulation)."""
    n = vflags.numel()
    _check("pf_coarsen_keys", lib.pf_coarsen_keys(_ptr(key), _ptr(vflags), n, int(levels), _ptr(key_out),
                                                  _ptr(vflags_out), _stream(stream)))


def query_multilevel(fine: Table, coarse: Table, slot, slot_coarse, r_in, g_in, b_in, vflags, vflags_coarse,
                     below: int, use_blend, r_out, g_out, b_out, count_out=None, stream=None):
    n = vflags.numel()
    _check("pf_query_multilevel", lib.pf_query_multilevel(
        fine.ref, coarse.ref, _ptr(slot), _ptr(slot_coarse), _ptr(r_in), _ptr(g_in), _ptr(b_in), _ptr(vflags),
        _ptr(vflags_coarse), n, int(below), int(bool(use_blend)), _ptr(r_out), _ptr(g_out), _ptr(b_out),
        _ptr(count_out), _stream(stream)))


MB_COPY, MB_GATHER, MB_SCATTER, MB_RMW, MB_CAS = 0, 1, 2, 3, 4
MB_THREADS = 2097152


def microbench(kind: int, buf, grain: int = 32, per_thread: int = 8, seed: int = 1, sink=None, stream=None):
    """One memory-system probe launch over the whole of `buf` (a device
    uint8 tensor, 256-byte aligned); returns the number of accesses made."""
    if sink is None:
        sink = torch.zeros(1, dtype=torch.int32, device=buf.device)
    _check("pf_microbench", lib.pf_microbench(kind, _ptr(buf), buf.numel(), grain, per_thread, seed, _ptr(sink),
                                              _stream(stream)))
    return buf.numel() // 2 if kind == MB_COPY else per_thread * MB_THREADS


def read_stats(t: Table, stream=None):
    import numpy as np
    out = np.zeros(STATS_LEN, np.uint64)
    _check("pf_read_stats", lib.pf_read_stats(t.ref, out.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
    return out


# ---------------------------------------------------------------- learned fallback
def geometry(key, px, py, pz, nx, ny, nz, cam):
    g = pf_geometry()
    g.key, g.px, g.py, g.pz = key.data_ptr(), px.data_ptr(), py.data_ptr(), pz.data_ptr()
    g.nx, g.ny, g.nz = nx.data_ptr(), ny.data_ptr(), nz.data_ptr()
    for c in range(3):
        g.cam[c] = float(cam[c])
    g._keep = (key, px, py, pz, nx, ny, nz)
    return g


class Mlp:
    """One network arena (a torch uint8 tensor) carved into the pf_mlp views."""

    def __init__(self, max_batch: int = 16384, device="cuda"):
        nbytes = int(lib.pf_mlp_bytes(max_batch))
        if nbytes == 0:
            raise PfError("pf_mlp_bytes", PF_ERANGE)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.m = pf_mlp()
        _check("pf_mlp_carve", lib.pf_mlp_carve(_ptr(self.arena), max_batch, ctypes.byref(self.m)))
        self.max_batch = max_batch
        self.steps = 0

    @property
    def ref(self):
        return ctypes.byref(self.m)

    def _view(self, addr, n, dtype, itemsize):
        off = addr - self.arena.data_ptr()
        return self.arena[off:off + n * itemsize].view(dtype)

    def weights(self) -> torch.Tensor:
        return self._view(self.m.w, MLP_NPARAM, torch.float32, 4)

    def weights_bf16(self) -> torch.Tensor:
        return self._view(self.m.wb, MLP_NPARAM, torch.int16, 2)

    def moments(self):
        return self._view(self.m.m, MLP_NPARAM, torch.float32, 4), self._view(self.m.v, MLP_NPARAM, torch.float32, 4)

    def partials(self, nblocks) -> torch.Tensor:
        return self._view(self.m.partial, nblocks * (MLP_NPARAM + 1), torch.float32, 4).view(nblocks, MLP_NPARAM + 1)

    def loss(self) -> torch.Tensor:
        return self._view(self.m.loss, 1, torch.float32, 4)


def mlp_init(m: Mlp, weights, stream=None):
    """Copies the FP32 weights in, then pf_mlp_init (moments to zero, BF16 copy)."""
    w = torch.as_tensor(weights, dtype=torch.float32).reshape(-1)
    m.weights().copy_(w.to(m.arena.device))
    m.steps = 0
    _check("pf_mlp_init", lib.pf_mlp_init(m.ref, _stream(stream)))


def mlp_select_workspace_bytes(n: int) -> int:
    return int(lib.pf_mlp_select_workspace_bytes(n))


def mlp_select(vflags, count, sparse_below, train_from, train_idx, sparse_idx, counts, workspace, stream=None):
    n = vflags.numel()
    _check("pf_mlp_select", lib.pf_mlp_select(_ptr(vflags), _ptr(count), n, sparse_below, train_from, _ptr(train_idx),
                                              _ptr(sparse_idx), _ptr(counts), _ptr(workspace), _stream(stream)))


def mlp_train_step(m: Mlp, t: Table, geo, slot, train_idx, counts, batch, seed, lr, step=None, stream=None):
    if step is None:
        m.steps += 1
        step = m.steps
    _check("pf_mlp_train_step", lib.pf_mlp_train_step(m.ref, t.ref, ctypes.byref(geo), _ptr(slot), _ptr(train_idx),
                                                      _ptr(counts), batch, int(seed) & 0xFFFFFFFFFFFFFFFF, step,
                                                      float(lr), _stream(stream)))


def mlp_features(geo, idx, out, stream=None):
    _check("pf_mlp_features", lib.pf_mlp_features(ctypes.byref(geo), _ptr(idx), idx.numel(), _ptr(out),
                                                  _stream(stream)))


def mlp_infer(m: Mlp, geo, sparse_idx, counts, r, g, b, stream=None):
    _check("pf_mlp_infer", lib.pf_mlp_infer(m.ref, ctypes.byref(geo), _ptr(sparse_idx), _ptr(counts),
                                            sparse_idx.numel(), _ptr(r), _ptr(g), _ptr(b), _stream(stream)))


# ---------------------------------------------------------------- many views
def views_workspace_bytes(ns, log2_slots) -> int:
    """Workspace bytes of pf_filter_views for views of ns[v] vertices and 2^log2_slots[v]-slot tables."""
    k = len(ns)
    return int(lib.pf_views_workspace_bytes((ctypes.c_uint64 * k)(*ns), (ctypes.c_uint32 * k)(*log2_slots), k))


def views_concurrent_workspace_bytes(ns, log2_slots) -> int:
    """Workspace bytes of pf_filter_views_concurrent."""
    k = len(ns)
    return int(lib.pf_views_concurrent_workspace_bytes((ctypes.c_uint64 * k)(*ns), (ctypes.c_uint32 * k)(*log2_slots),
                                                       k))


def filter_views_concurrent(descs, workspace, nstreams=1, stream=None):
    arr = (pf_view * len(descs))(*descs)
    _check("pf_filter_views_concurrent", lib.pf_filter_views_concurrent(
        arr, len(descs), nstreams, _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream)))


def make_view(f, key, vflags, slot, out, cur: Table, prev=None, count_out=None, temporal=True, alpha_old=0.2,
              idx_base=0):
    """Descriptor of one view; f holds px..nz, valid, r, g, b (device) and cam, s, seed."""
    d = pf_view()
    for name in ("px", "py", "pz", "nx", "ny", "nz", "r", "g", "b"):
        setattr(d, name, f[name].data_ptr())
    d.valid = f["valid"].data_ptr() if f.get("valid") is not None else None
    d.key = key.data_ptr() if key is not None else None
    d.vflags, d.slot = vflags.data_ptr(), slot.data_ptr()
    d.r_out, d.g_out, d.b_out = out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr()
    d.count_out = count_out.data_ptr() if count_out is not None else None
    d.cur = cur.t
    if prev is not None:
        d.prev = prev.t
    for c in range(3):
        d.kp.cam[c] = float(f["cam"][c])
    d.kp.s = float(f["s"])
    d.kp.seed = int(f["seed"]) & 0xFFFFFFFFFFFFFFFF
    d.kp.idx_base = int(idx_base)
    d.n = vflags.numel()
    d.alpha_old = float(alpha_old)
    d.temporal = int(bool(temporal))
    return d


def filter_views(descs, block, agg_width, workspace, grid_per_cu=0, stream=None):
    arr = (pf_view * len(descs))(*descs)
    _check("pf_filter_views", lib.pf_filter_views(arr, len(descs), block, agg_width, grid_per_cu, _ptr(workspace),
                                                  workspace.numel() * workspace.element_size(), _stream(stream)))
