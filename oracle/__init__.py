"""CPU oracle of hashed path space filtering -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library: the arithmetic is in
oracle/pf_oracle.c (plain C, built with gcc, fp-contract off) and the
MLP reference in oracle/mlp.py (numpy, float64).

filter_frame() composes the steps in the paper's order:
  keys (Algorithm 1) -> fixed-point radiance -> exact group-by on the key
  (Eq. (7)/(8), Section 3.2's gather form) -> linear-probing simulation
  (Section 3.2) -> average = sum / counter (Sections 3.2, 3.3.1) ->
  exponential moving average with the previous frame's set (Section 3.4.1),
  optionally followed by a low-density fallback (Section 3.3) or combined
  with a coarser level (multi-level accumulation, Section 3.3.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pf_oracle.c")
LIB = os.path.join(HERE, "libpf_oracle.so")
CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

INVALID, KEYRANGE, OVERFLOW, RADRANGE = 1, 2, 4, 8

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (x86-64 SSE, no contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        u64, u32, i32, f32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_float, ctypes.c_void_p
        L.orc_pcg32_outputs.argtypes = [u64, u64, u32, vp]
        L.orc_pcg32_first.argtypes = [u64, u64, vp]
        L.orc_fmix64.argtypes = [u64]; L.orc_fmix64.restype = u64
        L.orc_splitmix64.argtypes = [u64]; L.orc_splitmix64.restype = u64
        L.orc_level_of_detail.argtypes = [vp, f32, f32, f32]; L.orc_level_of_detail.restype = ctypes.c_int
        L.orc_build_keys.argtypes = [u64] + [vp] * 7 + [vp, f32, u64, u64, u32] + [vp] * 4 + [vp] * 3 + [i32]
        L.orc_quantize_radiance.argtypes = [u64, vp, vp, vp, i32, vp, vp]
        L.orc_group_by.argtypes = [u64, vp, vp, vp, vp, vp, vp, vp]; L.orc_group_by.restype = ctypes.c_int64
        L.orc_simulate_table.argtypes = [u64, vp, vp, vp, u32, u32, vp, vp, vp]
        L.orc_average.argtypes = [u64, vp, vp, i32, vp]
        L.orc_query.argtypes = [u64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_temporal_ema.argtypes = [u64, vp, vp, u64, vp, vp, f32, vp]
        L.orc_temporal_integrate.argtypes = [u64, vp, vp, vp, u64, vp, vp, vp, u32, vp, vp]
        L.orc_key_hashes.argtypes = [u64, vp, u32, vp, vp]
        L.orc_history_lookup.argtypes = [u64, vp, u32, vp, vp, vp, vp, vp]
        L.orc_history_update.argtypes = [u64, vp, vp, vp, u32, u32, u32, vp, vp, vp, vp]
        L.orc_low_density.argtypes = [u64, vp, vp, vp, vp, u32, ctypes.c_int, i32, vp, vp]
        L.orc_resolve_pixels.argtypes = [u64, u32, vp, vp, vp, ctypes.c_int, vp]
        L.orc_temporal_levels.argtypes = [u64, vp, vp, vp, u64, vp, vp, vp, ctypes.c_int, f32, u32, vp, vp, vp]
        L.orc_low_density.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a), dtype=np.float32)


# ---------------------------------------------------------------- primitives
def pcg32_outputs(initstate: int, initseq: int, count: int) -> np.ndarray:
    out = np.zeros(count, np.uint32)
    lib().orc_pcg32_outputs(initstate, initseq, count, _p(out))
    return out


def pcg32_first(initstate: int, n: int) -> np.ndarray:
    """First PCG32 output for streams 0..n-1 under one initial state."""
    out = np.zeros(max(n, 1), np.uint32)
    lib().orc_pcg32_first(initstate, n, _p(out))
    return out[:n].copy()


def fmix64(k: int) -> int:
    return int(lib().orc_fmix64(k))


def splitmix64(x: int) -> int:
    return int(lib().orc_splitmix64(x))


def level_of_detail(cam, x, y, z) -> int:
    c = _f32(cam)
    return int(lib().orc_level_of_detail(_p(c), float(np.float32(x)), float(np.float32(y)), float(np.float32(z))))


def build_keys(px, py, pz, nx, ny, nz, valid, cam, s, seed, idx_base, log2_slots, steps=False, level_up=0):
    """Key, fingerprint, home and flags per vertex (Algorithm 1); level_up > 0
    quantises the jittered position at level l' + level_up instead (the
    enclosing voxel of multi-level accumulation, Section 3.3.2)."""
    arrs = [_f32(a) for a in (px, py, pz, nx, ny, nz)]
    n = arrs[0].shape[0]
    v = None if valid is None else np.ascontiguousarray(valid, dtype=np.uint8)
    key = np.zeros(n, np.uint64); fp = np.zeros(n, np.uint32); home = np.zeros(n, np.uint32)
    flags = np.zeros(n, np.uint8)
    lvl = np.zeros(2 * n, np.int32) if steps else None
    xj = np.zeros(3 * n, np.float32) if steps else None
    xq = np.zeros(3 * n, np.int32) if steps else None
    camv = _f32(cam)
    lib().orc_build_keys(n, *[_p(a) for a in arrs], _p(v), _p(camv), float(np.float32(s)), seed, idx_base,
                         log2_slots, _p(key), _p(fp), _p(home), _p(flags), _p(lvl), _p(xj), _p(xq), int(level_up))
    out = {"key": key, "fp": fp, "home": home, "flags": flags}
    if steps:
        out["lvl"] = lvl.reshape(n, 2); out["xj"] = xj.reshape(n, 3); out["xq"] = xq.reshape(n, 3)
    return out


def quantize_radiance(r, g, b, frac_bits, flags):
    """int64 fixed point [n,3]; updates flags in place for unflagged vertices."""
    r, g, b = _f32(r), _f32(g), _f32(b)
    n = r.shape[0]
    q = np.zeros(3 * n, np.int64)
    lib().orc_quantize_radiance(n, _p(r), _p(g), _p(b), frac_bits, _p(flags), _p(q))
    return q.reshape(n, 3)


def group_by(key, flags, q):
    n = key.shape[0]
    gkey = np.zeros(max(n, 1), np.uint64); gcnt = np.zeros(max(n, 1), np.uint32)
    gsum = np.zeros(3 * max(n, 1), np.int64); vgroup = np.zeros(max(n, 1), np.int64)
    qq = np.ascontiguousarray(q, dtype=np.int64).reshape(-1)
    G = lib().orc_group_by(n, _p(np.ascontiguousarray(key, np.uint64)), _p(np.ascontiguousarray(flags, np.uint8)),
                           _p(qq), _p(gkey), _p(gcnt), _p(gsum), _p(vgroup))
    if G < 0:
        raise OverflowError("a cell sum leaves int64")
    return gkey[:G].copy(), gcnt[:G].copy(), gsum[:3 * G].reshape(G, 3).copy(), vgroup[:n].copy()


@dataclass
class TableSim:
    occupied: np.ndarray
    gslot: np.ndarray
    total_disp: int
    lmax: int
    alias: bool
    n_overflow: int
    hist: np.ndarray

    @property
    def order_free(self) -> bool:
        """True when every insertion order gives this exact outcome."""
        return not self.alias and self.n_overflow == 0


def simulate_table(gkey, gfp, ghome, log2_slots, max_probe) -> TableSim:
    G = gkey.shape[0]
    occ = np.zeros(1 << log2_slots, np.uint8)
    gslot = np.zeros(max(G, 1), np.int64)
    res = np.zeros(4 + 65, np.uint64)
    lib().orc_simulate_table(G, _p(np.ascontiguousarray(gkey, np.uint64)), _p(np.ascontiguousarray(gfp, np.uint32)),
                             _p(np.ascontiguousarray(ghome, np.uint32)), log2_slots, max_probe,
                             _p(occ), _p(gslot), _p(res))
    lmax = int(res[1])
    return TableSim(occ, gslot[:G].copy(), int(res[0]), lmax, bool(res[2]), int(res[3]), res[4:].copy())


def average(gcnt, gsum, frac_bits):
    G = gcnt.shape[0]
    out = np.zeros(3 * max(G, 1), np.float32)
    lib().orc_average(G, _p(np.ascontiguousarray(gcnt, np.uint32)), _p(np.ascontiguousarray(gsum, np.int64)),
                      frac_bits, _p(out))
    return out[:3 * G].reshape(G, 3).copy()


def temporal_ema(gkey, gnew, pkey, pold, alpha_old):
    G = gkey.shape[0]
    out = np.zeros(3 * max(G, 1), np.float32)
    pk = np.ascontiguousarray(pkey, np.uint64)
    assert np.all(pk[1:] > pk[:-1]), "previous keys must be strictly ascending"
    lib().orc_temporal_ema(G, _p(np.ascontiguousarray(gkey, np.uint64)), _p(_f32(gnew).reshape(-1)),
                           pk.shape[0], _p(pk), _p(_f32(pold).reshape(-1)), float(np.float32(alpha_old)), _p(out))
    return out[:3 * G].reshape(G, 3).copy()


def temporal_integrate(gkey, gnew, gcnt, pkey, pold, pcnt, max_samples):
    """Section 3.4.1's temporal integration with the sample-count threshold;
    returns (values [G,3] float32, stored counts [G] uint32)."""
    G = gkey.shape[0]
    out = np.zeros(3 * max(G, 1), np.float32)
    outn = np.zeros(max(G, 1), np.uint32)
    pk = np.ascontiguousarray(pkey, np.uint64)
    assert np.all(pk[1:] > pk[:-1]), "previous keys must be strictly ascending"
    lib().orc_temporal_integrate(G, _p(np.ascontiguousarray(gkey, np.uint64)), _p(_f32(gnew).reshape(-1)),
                                 _p(np.ascontiguousarray(gcnt, np.uint32)), pk.shape[0], _p(pk),
                                 _p(_f32(pold).reshape(-1)), _p(np.ascontiguousarray(pcnt, np.uint32)),
                                 int(max_samples), _p(out), _p(outn))
    return out[:3 * G].reshape(G, 3).copy(), outn[:G].copy()


CUBE, NORMALS = 0, 1  # low-density fallback modes


def low_density(gkey, gcnt, gsum, placed, gval, below, mode, frac_bits):
    """Section 3.3's fallbacks for voxels with fewer than `below` vertices:
    mode CUBE pools the 3x3x3 neighbourhood (same level and normal class),
    mode NORMALS the voxels at the same position and level with a similar
    normal class (positive dot product of the class vectors).  Returns
    (values [G,3] float32 with pooled voxels replaced, pooled mask [G])."""
    G = gkey.shape[0]
    out = np.ascontiguousarray(_f32(gval).reshape(-1)).copy()
    if out.shape[0] == 0:
        out = np.zeros(3, np.float32)
    pooled = np.zeros(max(G, 1), np.uint8)
    rc = lib().orc_low_density(G, _p(np.ascontiguousarray(gkey, np.uint64)), _p(np.ascontiguousarray(gcnt, np.uint32)),
                               _p(np.ascontiguousarray(gsum, np.int64).reshape(-1)),
                               _p(np.ascontiguousarray(placed, np.uint8)), int(below), int(mode), int(frac_bits),
                               _p(out), _p(pooled))
    if rc < 0:
        raise OverflowError("a pooled sum leaves int64")
    return out[:3 * G].reshape(G, 3).copy(), pooled[:G].astype(bool)


def temporal_levels(gkey, gnew, gcnt, pkey, pold, pcnt, mode, alpha_old, max_samples):
    """Section 3.4.2's changes of resolution across frames: the blend of
    temporal_ema (mode 0) / temporal_integrate (mode 1), with a voxel absent
    from the previous set taking its parent's value (N / 8 samples) or its
    children's count-weighted mean.  Returns (values [G,3], stored counts [G],
    how [G]: 0 none, 1 exact, 2 parent, 3 children)."""
    G = gkey.shape[0]
    out = np.zeros(3 * max(G, 1), np.float32)
    outn = np.zeros(max(G, 1), np.uint32)
    how = np.zeros(max(G, 1), np.uint8)
    pk = np.ascontiguousarray(pkey, np.uint64)
    assert np.all(pk[1:] > pk[:-1]), "previous keys must be strictly ascending"
    lib().orc_temporal_levels(G, _p(np.ascontiguousarray(gkey, np.uint64)), _p(_f32(gnew).reshape(-1)),
                              _p(np.ascontiguousarray(gcnt, np.uint32)), pk.shape[0], _p(pk),
                              _p(_f32(pold).reshape(-1)), _p(np.ascontiguousarray(pcnt, np.uint32)), int(mode),
                              float(np.float32(alpha_old)), int(max_samples), _p(out), _p(outn), _p(how))
    return out[:3 * G].reshape(G, 3).copy(), outn[:G].copy(), how[:G].copy()


@dataclass
class History:
    """Voxel values kept across frames with eviction by priority (Section
    3.4.3): direct-mapped, 2^log2 slots of (word, key, value (c, N), stamp);
    an empty slot has word = all ones.  See orc_history_update."""
    log2: int
    max_age: int
    word: np.ndarray
    key: np.ndarray
    val: np.ndarray
    stamp: np.ndarray

    @staticmethod
    def empty(log2: int, max_age: int) -> "History":
        m = 1 << log2
        return History(log2, max_age, np.full(m, np.iinfo(np.uint64).max, np.uint64), np.zeros(m, np.uint64),
                       np.zeros((m, 4), np.float32), np.zeros(m, np.uint32))

    def occupied(self) -> np.ndarray:
        return self.word != np.iinfo(np.uint64).max


def history_lookup(H: History, gkey):
    """(hit [G] bool, old [G,4] float32: c and N of the voxels found)."""
    G = gkey.shape[0]
    hit = np.zeros(max(G, 1), np.uint8)
    old = np.zeros(4 * max(G, 1), np.float32)
    lib().orc_history_lookup(G, _p(np.ascontiguousarray(gkey, np.uint64)), H.log2, _p(H.word), _p(H.key),
                             _p(H.val), _p(hit), _p(old))
    return hit[:G].astype(bool), old[:4 * G].reshape(G, 4).copy()


def history_update(H: History, gkey, gval, gn, frame: int):
    """Ages H to `frame` and lets this frame's voxels (values gval [G,3],
    counts gn) compete for their slots; updates H in place."""
    G = gkey.shape[0]
    lib().orc_history_update(G, _p(np.ascontiguousarray(gkey, np.uint64)), _p(_f32(gval).reshape(-1)),
                             _p(np.ascontiguousarray(gn, np.uint32)), H.log2, H.max_age, int(frame),
                             _p(H.word), _p(H.key), _p(H.val), _p(H.stamp))


def query(vgroup, gslot, gval, gcnt, r, g, b, flags):
    n = vgroup.shape[0]
    out = np.zeros(3 * max(n, 1), np.float32)
    cnt = np.zeros(max(n, 1), np.uint32)
    lib().orc_query(n, _p(np.ascontiguousarray(vgroup, np.int64)),
                    _p(None if gslot is None else np.ascontiguousarray(gslot, np.int64)),
                    _p(_f32(gval).reshape(-1)), _p(np.ascontiguousarray(gcnt, np.uint32)),
                    _p(_f32(r)), _p(_f32(g)), _p(_f32(b)), _p(out), _p(cnt), _p(flags))
    return out[:3 * n].reshape(n, 3).copy(), cnt[:n].copy()


# ---------------------------------------------------------------- one frame
@dataclass
class FrameResult:
    key: np.ndarray
    fp: np.ndarray
    home: np.ndarray
    flags: np.ndarray        # final flags (keys, radiance, overflow)
    q: np.ndarray            # [n,3] fixed point
    vgroup: np.ndarray
    gkey: np.ndarray         # distinct keys, ascending
    gfp: np.ndarray
    ghome: np.ndarray
    gcnt: np.ndarray
    gsum: np.ndarray         # [G,3] int64
    gavg: np.ndarray         # [G,3] float32
    gval: np.ndarray         # [G,3] value returned by lookup (blend when temporal)
    table: TableSim
    out: np.ndarray          # [n,3] per-vertex result
    cnt: np.ndarray          # [n] per-vertex cell count (0 when unfiltered)
    state: tuple             # (keys ascending, values, counts) of placed cells, for the next frame


def filter_frame(f: dict, cam=None, prev_state=None, alpha_old=0.2, temporal=True,
                 idx_base=0, s=None, seed=None, log2_slots=None, max_probe=None, frac_bits=None,
                 max_samples=None, low_density_fallback=None, level_up=0, history=None, frame=0,
                 across_levels=False):
    """The whole hot path for one view and frame on the CPU.

    f holds SoA arrays px..nz, r, g, b, valid (numpy or torch CPU) and the
    parameters cam, s, seed, log2_slots, max_probe, frac_bits (overridable).
    With temporal=True the lookup returns the moving average against
    prev_state (the state of the previous frame, None for the first frame),
    or, when max_samples is given, the temporal integration of Section 3.4.1
    with the stored sample count kept at most max_samples; the lookup's count
    is then the stored count.  low_density_fallback=(below, mode) then
    replaces the value of every placed voxel with fewer than `below` vertices
    in this frame by the pooled average of low_density(); the count the
    lookup returns is unchanged.  level_up > 0 filters with the voxels
    level_up levels coarser than each vertex's own (Section 3.3.2); a vertex
    flagged at its own level keeps that flag.  With a History (and
    temporal=True) the blend takes c_old from it instead of prev_state, and
    the frame's placed voxels then update it (history_update at `frame`).
    across_levels (with prev_state): temporal_levels, so that a voxel whose
    level changed finds its region one level coarser or finer.
    """
    A = {k: (v.numpy() if hasattr(v, "numpy") else v) for k, v in f.items() if k in
         ("px", "py", "pz", "nx", "ny", "nz", "r", "g", "b", "valid")}
    cam = f["cam"] if cam is None else cam
    s = f["s"] if s is None else s
    seed = f["seed"] if seed is None else seed
    m = f["log2_slots"] if log2_slots is None else log2_slots
    P = f["max_probe"] if max_probe is None else max_probe
    F = f["frac_bits"] if frac_bits is None else frac_bits

    k = build_keys(A["px"], A["py"], A["pz"], A["nx"], A["ny"], A["nz"], A["valid"], cam, s, seed, idx_base, m)
    if level_up:
        fine = k["flags"]
        k = build_keys(A["px"], A["py"], A["pz"], A["nx"], A["ny"], A["nz"], A["valid"], cam, s, seed, idx_base, m,
                       level_up=level_up)
        flagged = fine != 0
        k["flags"] = np.where(flagged, fine, k["flags"]).astype(np.uint8)
        for name in ("key", "fp", "home"):
            k[name] = np.where(flagged, 0, k[name]).astype(k[name].dtype)
    flags = k["flags"].copy()
    q = quantize_radiance(A["r"], A["g"], A["b"], F, flags)
    gkey, gcnt, gsum, vgroup = group_by(k["key"], flags, q)
    # fingerprint and home of each distinct key, taken from any of its vertices
    first = np.full(gkey.shape[0], -1, np.int64)
    idx = np.nonzero(vgroup >= 0)[0]
    first[vgroup[idx][::-1]] = idx[::-1]
    gfp = k["fp"][first] if gkey.shape[0] else np.zeros(0, np.uint32)
    ghome = k["home"][first] if gkey.shape[0] else np.zeros(0, np.uint32)
    sim = simulate_table(gkey, gfp, ghome, m, P)
    gavg = average(gcnt, gsum, F)
    placed = sim.gslot >= 0
    gn = gcnt
    if temporal and history is not None:
        pk = gkey[placed]
        hit, old = history_lookup(history, pk)
        if max_samples is None:
            gval = temporal_ema(gkey, gavg, pk[hit], old[hit][:, :3], alpha_old)
        else:
            gval, gn = temporal_integrate(gkey, gavg, gcnt, pk[hit], old[hit][:, :3],
                                          old[hit][:, 3].astype(np.uint32), max_samples)
        history_update(history, pk, gval[placed], gn[placed], frame)
    elif temporal and across_levels:
        pk, pv, pc = prev_state if prev_state is not None else (np.zeros(0, np.uint64), np.zeros((0, 3), np.float32),
                                                                np.zeros(0, np.uint32))
        gval, gn, _ = temporal_levels(gkey, gavg, gcnt, pk, pv, pc, 0 if max_samples is None else 1, alpha_old,
                                      (1 << 24) if max_samples is None else max_samples)
    elif temporal and max_samples is not None:
        pk, pv, pc = prev_state if prev_state is not None else (np.zeros(0, np.uint64), np.zeros((0, 3), np.float32),
                                                                np.zeros(0, np.uint32))
        gval, gn = temporal_integrate(gkey, gavg, gcnt, pk, pv, pc, max_samples)
    elif temporal and prev_state is not None:
        gval = temporal_ema(gkey, gavg, prev_state[0], prev_state[1], alpha_old)
    else:
        gval = gavg
    if low_density_fallback is not None:
        below, mode = low_density_fallback
        gval, _ = low_density(gkey, gcnt, gsum, placed, gval, below, mode, F)
    out, cnt = query(vgroup, sim.gslot, gval, gn, A["r"], A["g"], A["b"], flags)
    state = (gkey[placed].copy(), gval[placed].copy(), gn[placed].copy())
    return FrameResult(k["key"], k["fp"], k["home"], flags, q, vgroup, gkey, gfp, ghome, gcnt, gsum, gavg, gval,
                       sim, out, cnt, state)


def multilevel(fine: FrameResult, coarse: FrameResult, below: int):
    """Multi-level accumulation (Section 3.3.2): a vertex whose own voxel has
    fewer than `below` vertices (the lookup's count) takes its coarser
    voxel's value and count when that voxel was placed; otherwise its own
    voxel's.  Returns (out [n,3], count [n])."""
    use = (fine.flags == 0) & (fine.cnt < below) & (coarse.flags == 0)
    out = np.where(use[:, None], coarse.out, fine.out).astype(np.float32)
    cnt = np.where(use, coarse.cnt, fine.cnt).astype(np.uint32)
    return out, cnt


def resolve_pixels(out, throughput, valid, pixels: int, verts_per_path: int, init=None):
    """Section 3's resolve: per pixel, the sum over its path's vertices
    (bounce-major, vertex b of pixel p at b*pixels + p; those with valid != 0)
    of throughput * value, channel by channel in binary32, bounce 0 first;
    starting from init [pixels,3] when given.  out, throughput: [n,3]."""
    c3 = np.ascontiguousarray(_f32(out).reshape(-1))
    t3 = None if throughput is None else np.ascontiguousarray(_f32(throughput).reshape(-1))
    v = None if valid is None else np.ascontiguousarray(valid, dtype=np.uint8)
    px = np.zeros(3 * max(pixels, 1), np.float32) if init is None else np.ascontiguousarray(_f32(init).reshape(-1)).copy()
    lib().orc_resolve_pixels(pixels, verts_per_path, _p(c3), _p(t3), _p(v), int(init is not None), _p(px))
    return px[:3 * pixels].reshape(pixels, 3)


def key_hashes(key, log2_slots):
    """Home index and fingerprint of given keys (Algorithm 1's two hashes)."""
    k = np.ascontiguousarray(key, np.uint64)
    home = np.zeros(max(k.shape[0], 1), np.uint32); fp = np.zeros(max(k.shape[0], 1), np.uint32)
    lib().orc_key_hashes(k.shape[0], _p(k), log2_slots, _p(home), _p(fp))
    return home[:k.shape[0]].copy(), fp[:k.shape[0]].copy()


def filter_keys(key, r, g, b, valid, log2_slots, max_probe=64, frac_bits=24):
    """Accumulation, table simulation and lookup (no temporal blend) for a
    given key stream: Algorithm 1's hashes of each key, then the same steps
    as filter_frame after key construction."""
    key = np.ascontiguousarray(key, np.uint64)
    n = key.shape[0]
    home, fp = key_hashes(key, log2_slots)
    flags = np.where(np.asarray(valid) != 0, 0, INVALID).astype(np.uint8)
    q = quantize_radiance(r, g, b, frac_bits, flags)
    gkey, gcnt, gsum, vgroup = group_by(key, flags, q)
    G = gkey.shape[0]
    first = np.full(G, -1, np.int64)
    idx = np.nonzero(vgroup >= 0)[0]
    first[vgroup[idx][::-1]] = idx[::-1]
    gfp = fp[first] if G else np.zeros(0, np.uint32)
    ghome = home[first] if G else np.zeros(0, np.uint32)
    sim = simulate_table(gkey, gfp, ghome, log2_slots, max_probe)
    gavg = average(gcnt, gsum, frac_bits)
    out, cnt = query(vgroup, sim.gslot, gavg, gcnt, r, g, b, flags)
    return FrameResult(key, fp, home, flags, q, vgroup, gkey, gfp, ghome, gcnt, gsum, gavg, gavg, sim, out, cnt,
                       (gkey[sim.gslot >= 0].copy(), gavg[sim.gslot >= 0].copy(), gcnt[sim.gslot >= 0].copy()))


# ---------------------------------------------------- binary32 sums (variant)
@dataclass
class FloatFrameResult:
    key: np.ndarray
    flags: np.ndarray        # key flags, INVALID for non-finite contributions, OVERFLOW
    vgroup: np.ndarray
    gkey: np.ndarray
    gcnt: np.ndarray
    gsum: np.ndarray         # [G,3] float64 sums of the binary32 contributions
    gabs: np.ndarray         # [G,3] float64 sums of their magnitudes
    gmean: np.ndarray        # [G,3] float64 gsum / gcnt
    table: TableSim


def float_filter_frame(f: dict, cam=None, idx_base=0, s=None, seed=None, log2_slots=None, max_probe=None):
    """The accumulation as the paper performs it (Section 3.3.1: one
    floating-point atomic add per component of each vertex), reduced to what
    every arrival order shares: the partition of Eq. (7) is the same as
    filter_frame's, and each cell's mean (Eq. (8), w = 1) is taken over the
    binary32 contributions in float64 (rounding error at most n 2^-53 of
    the summed magnitudes, far below binary32's).  A GPU result in binary32
    may differ from gmean by the rounding of one float summation in some
    order plus one float division; the tests bound that from gabs.  No
    RADRANGE here: contributions are not scaled."""
    A = {k: (v.numpy() if hasattr(v, "numpy") else v) for k, v in f.items() if k in
         ("px", "py", "pz", "nx", "ny", "nz", "r", "g", "b", "valid")}
    cam = f["cam"] if cam is None else cam
    s = f["s"] if s is None else s
    seed = f["seed"] if seed is None else seed
    m = f["log2_slots"] if log2_slots is None else log2_slots
    P = f["max_probe"] if max_probe is None else max_probe
    k = build_keys(A["px"], A["py"], A["pz"], A["nx"], A["ny"], A["nz"], A["valid"], cam, s, seed, idx_base, m)
    flags = k["flags"].copy()
    rgb = [_f32(A[c]) for c in ("r", "g", "b")]
    finite = np.isfinite(rgb[0]) & np.isfinite(rgb[1]) & np.isfinite(rgb[2])
    flags[(flags == 0) & ~finite] = INVALID
    n = flags.shape[0]
    gkey, gcnt, _, vgroup = group_by(k["key"], flags, np.zeros((n, 3), np.int64))
    G = gkey.shape[0]
    first = np.full(G, -1, np.int64)
    idx = np.nonzero(vgroup >= 0)[0]
    first[vgroup[idx][::-1]] = idx[::-1]
    gfp = k["fp"][first] if G else np.zeros(0, np.uint32)
    ghome = k["home"][first] if G else np.zeros(0, np.uint32)
    sim = simulate_table(gkey, gfp, ghome, m, P)
    sel = vgroup >= 0
    gsum = np.zeros((G, 3)); gabs = np.zeros((G, 3))
    for c in range(3):
        x = rgb[c][sel].astype(np.float64)
        gsum[:, c] = np.bincount(vgroup[sel], weights=x, minlength=G)
        gabs[:, c] = np.bincount(vgroup[sel], weights=np.abs(x), minlength=G)
    gmean = gsum / np.maximum(gcnt, 1)[:, None].astype(np.float64)
    # vertices of keys the table could not place keep their own contribution
    lost = sel.copy()
    lost[sel] = sim.gslot[vgroup[sel]] < 0
    flags[lost] = OVERFLOW
    return FloatFrameResult(k["key"], flags, vgroup, gkey, gcnt, gsum, gabs, gmean, sim)
