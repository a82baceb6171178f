"""The C ABI on a host without a GPU: the library loads, exports every entry
point include/pf.h declares, and its host-side argument checks return the
documented status before anything is launched."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pf.h")).read()
    return sorted(set(re.findall(r"^\s*(?:pf_status|size_t|uint64_t|const char \*)\s*(pf_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def pf():
    import paper_1902_05942_amd as pf
    return pf


def test_every_declared_symbol_is_exported(pf):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(pf._lib.lib, n), n
    assert set(names) == set(pf._lib.EXPORTED)


def test_struct_layouts_match_header(pf):
    assert ctypes.sizeof(pf._lib.pf_table) == 5 * 8 + 4 * 4
    assert ctypes.sizeof(pf._lib.pf_key_params) == 4 * 4 + 8 + 8
    assert ctypes.sizeof(pf._lib.pf_view) == 296
    assert ctypes.sizeof(pf._lib.pf_mlp) == 6 * 8 + 8
    assert ctypes.sizeof(pf._lib.pf_geometry) == 7 * 8 + 16
    assert pf._lib.CELL_BYTES == 32


def test_table_sizing_and_carving(pf):
    L = pf._lib.lib
    assert L.pf_table_bytes(3, 1) == 0 and L.pf_table_bytes(31, 1) == 0
    b22 = L.pf_table_bytes(22, 1)
    S = 1 << 22
    assert b22 >= S * 64 + S // 8                # 64-byte slot records and the bitmap
    assert L.pf_table_bytes(22, 0) == b22         # the records keep the temporal value's space
    t = pf._lib.pf_table()
    base = 0x7F0000000010                       # never dereferenced: carving is arithmetic
    assert L.pf_table_carve(ctypes.c_void_p(base), 22, 1, 64, 24, ctypes.byref(t)) == 0
    assert t.cell % 256 == 0 and t.cell >= base and t.stats + 128 * 8 <= base + b22
    assert t.key - t.cell == 32 and t.blend - t.cell == 48   # fields of slot 0, stride 64
    assert pf._lib.SLOT_BYTES == 64
    t0 = pf._lib.pf_table()
    assert L.pf_table_carve(ctypes.c_void_p(base), 22, 0, 64, 24, ctypes.byref(t0)) == 0 and not t0.blend
    for bad in [(3, 64, 24), (31, 64, 24), (10, 0, 24), (10, 1025, 24), (10, 64, 7), (10, 64, 41)]:
        assert L.pf_table_carve(ctypes.c_void_p(base), bad[0], 1, bad[1], bad[2], ctypes.byref(t)) == pf._lib.PF_ERANGE
    assert L.pf_table_carve(None, 10, 1, 64, 24, ctypes.byref(t)) == pf._lib.PF_EINVAL


def test_argument_checks_return_before_launch(pf):
    L, lp = pf._lib.lib, pf._lib
    t = lp.pf_table()
    assert L.pf_table_carve(ctypes.c_void_p(0x7F0000000000), 10, 1, 64, 24, ctypes.byref(t)) == 0
    kp = lp.pf_key_params()
    kp.s = 0.01
    fake = ctypes.c_void_p(0x7F0000100000)
    # n == 0 is a no-op
    assert L.pf_build_keys(*([None] * 7), 0, ctypes.byref(kp), 10, None, None, None, None, None) == lp.PF_OK
    assert L.pf_insert_accumulate(ctypes.byref(t), None, None, None, None, None, None, 0, 0, None) == lp.PF_OK
    assert L.pf_query_average(ctypes.byref(t), None, None, None, None, None, None, 0, 0, None, None, None, None,
                              None) == lp.PF_OK
    # NULL and misaligned pointers
    assert L.pf_build_keys(*([None] * 7), 5, ctypes.byref(kp), 10, None, None, None, None, None) == lp.PF_EINVAL
    assert L.pf_build_keys(*([fake] * 6), None, 5, None, 10, fake, None, None, fake, None) == lp.PF_EINVAL
    odd = ctypes.c_void_p(0x7F0000100002)
    assert L.pf_build_keys(odd, *([fake] * 5), None, 5, ctypes.byref(kp), 10, fake, None, None, fake,
                           None) == lp.PF_EINVAL
    assert L.pf_insert_accumulate(ctypes.byref(t), fake, fake, fake, None, fake, None, 5, 0, None) == lp.PF_EINVAL
    assert L.pf_query_average(ctypes.byref(t), None, None, fake, fake, fake, fake, 5, 0, fake, fake, fake, None,
                              None) == lp.PF_EINVAL
    # parameter ranges
    kp.s = 0.0
    assert L.pf_build_keys(*([fake] * 6), None, 5, ctypes.byref(kp), 10, fake, None, None, fake,
                           None) == lp.PF_ERANGE
    kp.s = float("nan")
    assert L.pf_build_keys(*([fake] * 6), None, 5, ctypes.byref(kp), 10, fake, None, None, fake,
                           None) == lp.PF_ERANGE
    kp.s = 0.01
    assert L.pf_build_keys(*([fake] * 6), None, 5, ctypes.byref(kp), 31, fake, None, None, fake,
                           None) == lp.PF_ERANGE
    assert L.pf_insert_accumulate(ctypes.byref(t), fake, fake, fake, fake, fake, None, 5, 3, None) == lp.PF_ERANGE
    assert L.pf_insert_accumulate(ctypes.byref(t), fake, fake, fake, fake, fake, None, 5, 512, None) == lp.PF_ERANGE
    assert L.pf_insert_accumulate(ctypes.byref(t), fake, fake, fake, fake, fake, None, 1 << 32, 0,
                                  None) == lp.PF_EINVAL
    # launch sizes are computed in 32 bits: n is limited to 2^31
    assert L.pf_build_keys(*([fake] * 6), None, (1 << 31) + 1, ctypes.byref(kp), 10, fake, None, None, fake,
                           None) == lp.PF_EINVAL
    assert L.pf_query_average(ctypes.byref(t), fake, None, fake, fake, fake, fake, (1 << 31) + 1, 0, fake, fake,
                              fake, None, None) == lp.PF_EINVAL
    assert L.pf_temporal_update(ctypes.byref(t), None, ctypes.c_float(1.5), 0, None) == lp.PF_ERANGE
    assert L.pf_temporal_update(ctypes.byref(t), None, ctypes.c_float(0.2), 7, None) == lp.PF_ERANGE
    assert L.pf_temporal_integrate(ctypes.byref(t), None, 0, None) == lp.PF_ERANGE
    assert L.pf_temporal_integrate(ctypes.byref(t), None, (1 << 24) + 1, None) == lp.PF_ERANGE
    t2 = lp.pf_table()
    assert L.pf_table_carve(ctypes.c_void_p(0x7E0000000000), 11, 1, 64, 24, ctypes.byref(t2)) == 0
    assert L.pf_temporal_update(ctypes.byref(t), ctypes.byref(t2), ctypes.c_float(0.2), 0, None) == lp.PF_ERANGE
    t3 = lp.pf_table()
    assert L.pf_table_carve(ctypes.c_void_p(0x7D0000000000), 10, 0, 64, 24, ctypes.byref(t3)) == 0
    assert L.pf_temporal_update(ctypes.byref(t3), None, ctypes.c_float(0.2), 0, None) == lp.PF_EINVAL
    assert L.pf_query_average(ctypes.byref(t3), fake, None, fake, fake, fake, fake, 5, 1, fake, fake, fake, None,
                              None) == lp.PF_EINVAL
    # the lookup with the clear of another table: that table is required and
    # its slots may not overlap the looked-up table's
    qc = L.pf_query_average_clear
    assert qc(ctypes.byref(t), fake, None, fake, fake, fake, fake, 5, 0, fake, fake, fake, None, None,
              None) == lp.PF_EINVAL
    assert qc(ctypes.byref(t), fake, None, fake, fake, fake, fake, 5, 0, fake, fake, fake, None, ctypes.byref(t),
              None) == lp.PF_EINVAL
    t4 = lp.pf_table()   # starts inside t's slot records
    assert L.pf_table_carve(ctypes.c_void_p(0x7F0000000000 + 256 * 64), 10, 1, 64, 24, ctypes.byref(t4)) == 0
    assert qc(ctypes.byref(t), fake, None, fake, fake, fake, fake, 5, 0, fake, fake, fake, None, ctypes.byref(t4),
              None) == lp.PF_EINVAL
    assert qc(ctypes.byref(t3), fake, None, fake, fake, fake, fake, 5, 1, fake, fake, fake, None, ctypes.byref(t2),
              None) == lp.PF_EINVAL   # no temporal values to look up
    assert qc(ctypes.byref(t), None, None, fake, fake, fake, fake, 5, 0, fake, fake, fake, None, ctypes.byref(t2),
              None) == lp.PF_EINVAL   # neither key nor slot
    # the insert with the temporal pass in it: the checks of the insert, then
    # those of the temporal pass, all before any launch
    kt = L.pf_build_keys_insert_binned_temporal
    big = 1 << 40

    def kit(cur, prev, alpha=0.2, max_samples=0, s=0.01):
        kp.s = s
        return kt(ctypes.byref(cur), *([fake] * 6), None, ctypes.byref(kp), fake, fake, fake, 5, None, fake, fake,
                  fake, big, None if prev is None else ctypes.byref(prev), ctypes.c_float(alpha), max_samples, None)
    t5 = lp.pf_table()
    assert L.pf_table_carve(ctypes.c_void_p(0x7C0000000000), 10, 1, 64, 24, ctypes.byref(t5)) == 0
    assert kit(t, t5, s=0.0) == lp.PF_ERANGE                       # the insert's own checks come first
    assert kit(t3, None) == lp.PF_EINVAL                           # no temporal values in t
    assert kit(t, t3) == lp.PF_EINVAL                              # nor in prev
    assert kit(t, t) == lp.PF_EINVAL                               # prev is t
    assert kit(t, t2) == lp.PF_ERANGE                              # log2_slots differ
    assert kit(t, t5, alpha=1.5) == lp.PF_ERANGE
    assert kit(t, t5, max_samples=(1 << 24) + 1) == lp.PF_ERANGE
    kp.s = 0.01
    # low-density fallback: needs the blend array and fixed-point sums, a known mode; below <= 1 is a no-op
    assert L.pf_low_density_fallback(ctypes.byref(t3), 4, 0, None) == lp.PF_EINVAL
    assert L.pf_low_density_fallback(ctypes.byref(t), 4, 2, None) == lp.PF_ERANGE
    assert L.pf_low_density_fallback(ctypes.byref(t), 1, 0, None) == lp.PF_OK
    assert L.pf_low_density_fallback(None, 4, 0, None) == lp.PF_EINVAL
    # pixel resolve: arrays, throughput all or none, size limit
    assert L.pf_resolve_pixels(*([None] * 7), 0, 3, 0, None, None, None, None) == lp.PF_OK
    assert L.pf_resolve_pixels(fake, fake, fake, fake, None, None, None, 5, 3, 0, fake, fake, fake, None) == \
        lp.PF_EINVAL
    assert L.pf_resolve_pixels(fake, fake, fake, None, None, None, None, 5, 3, 0, None, fake, fake, None) == \
        lp.PF_EINVAL
    assert L.pf_resolve_pixels(fake, fake, fake, None, None, None, None, 1 << 30, 3, 0, fake, fake, fake,
                               None) == lp.PF_EINVAL
    # history: sizes, arrays, modes
    assert L.pf_history_bytes(3) == 0 and L.pf_history_bytes(31) == 0
    assert L.pf_history_bytes(10) >= (1 << 10) * 36
    h = lp.pf_history()
    assert L.pf_history_carve(ctypes.c_void_p(0x7C0000000000), 10, 3, ctypes.byref(h)) == lp.PF_OK
    assert L.pf_history_carve(ctypes.c_void_p(0x7C0000000000), 31, 3, ctypes.byref(h)) == lp.PF_ERANGE
    assert L.pf_history_init(None, None) == lp.PF_EINVAL
    assert L.pf_temporal_history(ctypes.byref(t), None, ctypes.c_float(0.2), 0, 1, 0, None) == lp.PF_EINVAL
    assert L.pf_temporal_history(ctypes.byref(t3), ctypes.byref(h), ctypes.c_float(0.2), 0, 1, 0, None) == \
        lp.PF_EINVAL
    assert L.pf_temporal_history(ctypes.byref(t), ctypes.byref(h), ctypes.c_float(0.2), 2, 1, 0, None) == \
        lp.PF_ERANGE
    assert L.pf_temporal_history(ctypes.byref(t), ctypes.byref(h), ctypes.c_float(0.2), 1, 0, 0, None) == \
        lp.PF_ERANGE
    # multi-level: levels in [1, 31], arrays required, blend arrays with use_blend
    assert L.pf_coarsen_keys(fake, fake, 5, 0, fake, fake, None) == lp.PF_ERANGE
    assert L.pf_coarsen_keys(fake, fake, 5, 32, fake, fake, None) == lp.PF_ERANGE
    assert L.pf_coarsen_keys(None, fake, 5, 1, fake, fake, None) == lp.PF_EINVAL
    assert L.pf_coarsen_keys(None, None, 0, 1, None, None, None) == lp.PF_OK
    assert L.pf_query_multilevel(ctypes.byref(t), ctypes.byref(t), fake, None, fake, fake, fake, fake, fake, 5, 4, 0,
                                 fake, fake, fake, None, None) == lp.PF_EINVAL
    assert L.pf_query_multilevel(ctypes.byref(t), ctypes.byref(t3), fake, fake, fake, fake, fake, fake, fake, 5, 4, 1,
                                 fake, fake, fake, None, None) == lp.PF_EINVAL
    # binary32 sums: accepted by the atomic insert's checks, refused by the binned insert; unknown formats refused
    tf = lp.pf_table()
    assert L.pf_table_carve(ctypes.c_void_p(0x7C0000000000), 10, 1, 64, 24, ctypes.byref(tf)) == 0
    assert tf.sum_format == lp.SUMS_FIXED64
    tf.sum_format = lp.SUMS_FLOAT32
    assert L.pf_insert_accumulate(ctypes.byref(tf), fake, fake, fake, None, fake, None, 5, 0, None) == lp.PF_EINVAL
    assert L.pf_insert_accumulate(ctypes.byref(tf), fake, fake, fake, fake, fake, None, 5, 3, None) == lp.PF_ERANGE
    assert L.pf_insert_accumulate_binned(ctypes.byref(tf), fake, fake, fake, fake, fake, fake, 5, fake, 1 << 30,
                                         None) == lp.PF_EINVAL
    tf.sum_format = 2
    assert L.pf_clear(ctypes.byref(tf), None) == lp.PF_EINVAL
    # memory-system probe: kinds, granules and footprints are checked before any launch
    buf = ctypes.c_void_p(0x7B0000000000)
    assert L.pf_microbench(9, buf, 1 << 20, 32, 1, 1, fake, None) == lp.PF_ERANGE
    assert L.pf_microbench(lp.MB_GATHER, buf, 1 << 20, 24, 1, 1, fake, None) == lp.PF_ERANGE
    assert L.pf_microbench(lp.MB_RMW, buf, 1 << 20, 16, 1, 1, fake, None) == lp.PF_ERANGE
    assert L.pf_microbench(lp.MB_GATHER, buf, 3 << 20, 32, 1, 1, fake, None) == lp.PF_ERANGE
    assert L.pf_microbench(lp.MB_GATHER, buf, 1 << 20, 32, 0, 1, fake, None) == lp.PF_ERANGE
    assert L.pf_microbench(lp.MB_GATHER, ctypes.c_void_p(0x7B0000000010), 1 << 20, 32, 1, 1, fake,
                           None) == lp.PF_EINVAL
    assert L.pf_microbench(lp.MB_COPY, buf, 48, 32, 1, 1, fake, None) == lp.PF_ERANGE
    # a corrupted table descriptor
    t.log2_slots = 40
    assert L.pf_clear(ctypes.byref(t), None) == lp.PF_ERANGE
    assert L.pf_clear(None, None) == lp.PF_EINVAL
    assert L.pf_read_stats(None, None, None) == lp.PF_EINVAL


def test_product_path_has_no_fallback(pf):
    """The package loads libpf.so and nothing else; without it, import fails."""
    import subprocess
    import sys
    code = ("import os, sys; sys.path.insert(0, %r); import paper_1902_05942_amd._lib as L; "
            "print(L.LIB_PATH)") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip().endswith("libpf.so")
    src = open(os.path.join(ROOT, "paper_1902_05942_amd", "__init__.py")).read()
    src += open(os.path.join(ROOT, "paper_1902_05942_amd", "_lib.py")).read()
    assert "oracle" not in src
