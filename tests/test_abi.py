"""The C-ABI library without a GPU: it loads, exports every symbol the header
declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def msf():
    import paper_2302_12199_amd as msf
    if not os.path.exists(msf.LIB_PATH):
        pytest.fail("libmsf.so not built: run __graft_entry__.build()")
    return msf


def declared_functions():
    text = open(os.path.join(ROOT, "include", "msf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\**\s+\**(msf_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol(msf):
    names = declared_functions()
    assert names, "no declarations parsed"
    assert sorted(msf.SYMBOLS) == names
    lib = msf.library()
    for name in names:
        assert getattr(lib, name) is not None


def test_status_strings(msf):
    lib = msf.library()
    assert lib.msf_status_string(0) == b"ok"
    assert lib.msf_status_string(msf.ERANGE) == b"vertex id out of range"
    assert lib.msf_version() >= 100


def test_workspace_size_monotone(msf):
    a = msf.workspace_bytes(1000, 100)
    b = msf.workspace_bytes(2000, 100)
    c = msf.workspace_bytes(2000, 200)
    assert 0 < a < b < c
    assert msf.workspace_bytes(2**28, 2**24) > 32 * 2**28


FAKE = 0x1000  # never dereferenced: argument checks run before any device work


@pytest.mark.parametrize("m,n", [(-1, 5), (5, -1), (2**32, 5), (5, 2**31), (3, 0)])
def test_rejects_bad_sizes(msf, m, n):
    rc, _ = msf.compute_raw(FAKE, FAKE, FAKE, m, n, FAKE)
    assert rc == msf.EINVAL


def test_rejects_null_pointers(msf):
    for args in [(0, FAKE, FAKE, FAKE), (FAKE, 0, FAKE, FAKE), (FAKE, FAKE, 0, FAKE),
                 (FAKE, FAKE, FAKE, 0)]:
        rc, _ = msf.compute_raw(args[0], args[1], args[2], 10, 5, args[3])
        assert rc == msf.EINVAL
    total = ctypes.c_uint64()
    rc = msf.library().msf_compute(FAKE, FAKE, FAKE, 10, 5, FAKE, None, None, 0, None, None, None)
    assert rc == msf.EINVAL


def test_rejects_bad_options(msf):
    for kw in [dict(algo=7), dict(pivot=9), dict(quantile=1.5), dict(quantile=float("nan")),
               dict(sample_size=-1), dict(round0=3), dict(round0=-1),
               dict(tail_threshold=-1), dict(tail_threshold=1025)]:
        rc, _ = msf.compute_raw(FAKE, FAKE, FAKE, 10, 5, FAKE, options=msf.make_options(**kw))
        assert rc == msf.EINVAL, kw
    o = msf.make_options()
    o.reserved[2] = 1
    assert msf.compute_raw(FAKE, FAKE, FAKE, 10, 5, FAKE, options=o)[0] == msf.EINVAL


def test_workspace_sizes_of_the_round0_choices(msf):
    # the bucketed round 0 needs about 24 B per edge and 8 B per vertex more,
    # only where it applies
    m, n = 1 << 22, 1 << 21
    auto, edges = msf.workspace_bytes(m, n), msf.workspace_bytes(m, n, round0="edges")
    assert auto == msf.workspace_bytes(m, n, round0="buckets")
    assert 24 * m + 8 * n <= auto - edges <= 26 * m + 9 * n + (1 << 20)
    for m, n in [(1 << 20, 1 << 16), ((1 << 22) - 1, 1 << 21), (1 << 22, (1 << 21) - 1),
                 (1 << 22, (1 << 24) + 1)]:   # too small or too many vertices
        assert msf.workspace_bytes(m, n) == msf.workspace_bytes(m, n, round0="edges")
    for algo in ["boruvka", "filter"]:
        assert msf.workspace_bytes(1 << 28, 1 << 24, algo=algo) > \
            msf.workspace_bytes(1 << 28, 1 << 24, algo=algo, round0="edges")


def test_workspace_too_small(msf):
    need = msf.workspace_bytes(10, 5)
    rc, _ = msf.compute_raw(FAKE, FAKE, FAKE, 10, 5, FAKE, workspace_ptr=FAKE,
                            workspace_bytes=need - 1)
    assert rc == msf.EWORKSPACE


def test_workspace_not_256_byte_aligned(msf):
    need = msf.workspace_bytes(10, 5)
    rc, _ = msf.compute_raw(FAKE, FAKE, FAKE, 10, 5, FAKE, workspace_ptr=FAKE + 16,
                            workspace_bytes=need)
    assert rc == msf.EINVAL


def test_allocation_failure_is_reported(msf):
    # no workspace given: the library allocates one, which fails without a
    # usable device (this test runs on the CPU) -> MSF_ENOMEM, nothing launched
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present: the allocation would succeed")
    rc, _ = msf.compute_raw(FAKE, FAKE, FAKE, 10, 5, FAKE)
    assert rc == msf.ENOMEM


def test_empty_graph_needs_no_device(msf):
    st = msf.Stats()
    rc, total = msf.compute_raw(0, 0, 0, 0, 7, 0, stats=st)
    assert rc == msf.OK and total == 0 and st.msf_edges == 0


def test_no_cpu_fallback(msf, monkeypatch, tmp_path):
    import importlib
    import sys
    monkeypatch.setattr(msf, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(msf, "_LIB", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        msf.library()


def test_batched_argument_checks(msf):
    lib = msf.library()
    o = msf.make_batch_options(block=300)
    rc = lib.msf_compute_batched(FAKE, FAKE, FAKE, FAKE, FAKE, 3, 10, None, FAKE, FAKE, None,
                                 FAKE, 1 << 30, None, ctypes.byref(o))
    assert rc == msf.EINVAL
    rc = lib.msf_compute_batched(FAKE, FAKE, FAKE, FAKE, FAKE, -1, 10, None, FAKE, FAKE, None,
                                 FAKE, 1 << 30, None, None)
    assert rc == msf.EINVAL
    rc = lib.msf_compute_batched(FAKE, FAKE, FAKE, FAKE, FAKE, 3, 10, None, FAKE, FAKE, None,
                                 FAKE, 16, None, None)
    assert rc == msf.EWORKSPACE
    rc = lib.msf_compute_batched(FAKE, FAKE, FAKE, FAKE, FAKE, 3, 10, None, FAKE, FAKE, None,
                                 FAKE + 16, 1 << 30, None, None)
    assert rc == msf.EINVAL                      # workspace not 256-byte aligned
    for kw in (dict(wave_min=1), dict(wave_min=65), dict(hot_min=65), dict(hot_min=-2),
               dict(wave_edges=-2), dict(wave_edges=4096)):   # the wave tier is switched off
        o = msf.make_batch_options(**kw)
        assert lib.msf_compute_batched(FAKE, FAKE, FAKE, FAKE, FAKE, 3, 10, None, FAKE, FAKE,
                                       None, FAKE, 1 << 30, None, ctypes.byref(o)) == msf.EINVAL
    o = msf.make_batch_options()
    o.reserved[0] = 1
    assert lib.msf_compute_batched(FAKE, FAKE, FAKE, FAKE, FAKE, 3, 10, None, FAKE, FAKE, None,
                                   FAKE, 1 << 30, None, ctypes.byref(o)) == msf.EINVAL
    # an empty batch needs no device
    assert lib.msf_compute_batched(None, None, None, None, None, 0, 0, None, None, None, None,
                                   None, 0, None, None) == msf.OK


def test_noalloc_argument_checks_before_the_device(msf):
    lib = msf.library()
    total = ctypes.c_uint64(0)
    # beyond the static scratch: rejected before any device call
    m, n = 4 << 20, 1 << 20
    assert msf.workspace_bytes(m, n) > msf.NOALLOC_SCRATCH_BYTES
    rc = lib.msf_compute_noalloc(FAKE, FAKE, FAKE, m, n, FAKE, ctypes.byref(total), None, None,
                                 None)
    assert rc == msf.EWORKSPACE
    assert b"static scratch" in lib.msf_last_error()
    assert lib.msf_compute_noalloc(FAKE, FAKE, FAKE, 10, 0, FAKE, ctypes.byref(total), None,
                                   None, None) == msf.EINVAL
    assert lib.msf_compute_noalloc(FAKE, 0, FAKE, 10, 5, FAKE, ctypes.byref(total), None,
                                   None, None) == msf.EINVAL
    o = msf.make_options(quantile=2.0)
    assert lib.msf_compute_noalloc(FAKE, FAKE, FAKE, 10, 5, FAKE, ctypes.byref(total), None,
                                   ctypes.byref(o), None) == msf.EINVAL
    st = msf.Stats()
    assert lib.msf_compute_noalloc(None, None, None, 0, 3, None, ctypes.byref(total), None,
                                   None, ctypes.byref(st)) == msf.OK
    assert total.value == 0 and st.base_cases == 1
    # the scratch size in the binding is the header's
    text = open(os.path.join(ROOT, "include", "msf.h")).read()
    assert "#define MSF_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)" in text
    assert msf.NOALLOC_SCRATCH_BYTES == 128 << 20
