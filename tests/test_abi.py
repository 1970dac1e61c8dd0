"""Host-side checks of the C ABI (CPU only: the library loads and exports what iht.h declares)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iht.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(iht_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_1608_01398_amd import iht

    if not os.path.exists(iht.LIB_PATH):
        from paper_1608_01398_amd import build

        build.build()
    return iht.LIB_PATH


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ("iht_fit", "iht_gradient", "iht_project", "iht_geno_create", "iht_stats_create"):
        assert f in fns


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.check_output(["nm", "-D", "--defined-only", lib_path], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    from paper_1608_01398_amd import iht

    assert set(iht.EXPORTS) == set(declared_functions())


def test_library_loads_and_answers_host_only_calls(lib_path):
    from paper_1608_01398_amd import iht

    L = iht.load()
    o = iht.default_opts()
    assert o.max_iter == 200 and o.max_backtrack == 50 and abs(o.c - 0.01) < 1e-15 and o.shrink == 0.5
    assert o.tol == 1e-10 and o.precision == iht.FP64
    assert L.iht_status_str(iht.STALLED).decode().startswith("stalled")
    # argument validation returns before touching the device
    h = ctypes.c_void_p()
    rc = L.iht_geno_create(None, 10, 10, 3, 0, None, ctypes.byref(h))
    assert rc == iht.EINVAL and b"NULL" in L.iht_last_error()
    buf = (ctypes.c_uint8 * 30)()
    rc = L.iht_geno_create(ctypes.cast(buf, ctypes.c_void_p), 10, 10, 2, 0, None, ctypes.byref(h))
    assert rc == iht.EINVAL and b"row_bytes" in L.iht_last_error()
    # size limits: a tile's packed bytes stay addressable with 32-bit offsets
    for n, p in ((10, (1 << 28) - 8192 + 1), ((1 << 24) + 1, 10), (0, 10), (10, 0)):
        rc = L.iht_geno_create(ctypes.cast(buf, ctypes.c_void_p), n, p, 3, 0, None, ctypes.byref(h))
        assert rc == iht.EINVAL and b"out of range" in L.iht_last_error(), (n, p)
    rc = L.iht_project(None, 10, 3, None, None, None)
    assert rc == iht.EINVAL
    assert L.iht_fit(None, None, None, None, 0, 1, 3, None, None, None, None, None, None, None) == iht.EINVAL
    # the server entry points reject NULL handles before any device work
    srv = ctypes.c_void_p()
    assert L.iht_server_create(None, 4, 10, 1 << 30, None, 0, 1, None, None, ctypes.byref(srv)) == iht.EINVAL
    assert srv.value is None
    done = ctypes.c_int32(7)
    assert L.iht_server_step(None, ctypes.byref(done)) == iht.EINVAL
    assert L.iht_server_poll(None, 0, ctypes.byref(done)) == iht.EINVAL
    info = iht.ServerInfo()
    assert L.iht_server_info(None, ctypes.byref(info)) == iht.EINVAL
    rid = ctypes.c_int64(0)
    assert L.iht_server_submit(None, None, None, 0, 1, None, None, None, None, None, None, None,
                               ctypes.byref(rid)) == iht.EINVAL
    assert L.iht_server_destroy(None) == iht.OK


def test_oracle_builds_and_is_not_linked_by_the_library(lib_path):
    from oracle import oracle

    oracle.build(force=False)
    out = subprocess.check_output(["ldd", lib_path], text=True)
    assert "oracle" not in out
    deps = subprocess.check_output(["nm", "-D", "--undefined-only", lib_path], text=True)
    assert "iht_ref" not in deps


def test_workspace_bytes_host_only(lib_path):
    """iht_workspace_bytes sizes the caller's workspace on the host (no device needed): it grows
    linearly with the number of solves, with the model size and (per solve) with p; the matrix-core
    path needs more (its residual digits and scales); one fit equals a batch of one; arguments out of
    range give 0."""
    from paper_1608_01398_amd import iht

    one = iht.workspace_bytes(5000, 500_000, 20, 1, iht.FP64)
    assert one > 0 and one % 256 == 0
    assert one == iht.workspace_bytes(5000, 500_000, 20, 1, iht.FP64, T=1)
    # per solve: beta and g (16 B per SNP) and the top-k candidates (12 B per SNP) dominate at this
    # shape; beside them one fixed area (the split pass's partial sums) serves every solve
    per = iht.workspace_bytes(5000, 500_000, 20, 1, iht.FP64, T=2) - one
    assert 28 * 500_000 <= per <= 28 * 500_000 + (4 << 20)
    assert one >= per
    eight = iht.workspace_bytes(5000, 500_000, 20, 1, iht.FP64, T=8)
    assert abs(eight - one - 7 * per) <= 7 * 40 * 256  # linear in T up to the 256-byte alignment of ~40 buffers
    assert iht.workspace_bytes(5000, 500_000, 40, 1, iht.FP64) > one
    # the per-solve part grows with p (the fixed part follows the pass geometry, which p also sets)
    per_600k = (iht.workspace_bytes(5000, 600_000, 20, 1, iht.FP64, T=2)
                - iht.workspace_bytes(5000, 600_000, 20, 1, iht.FP64))
    assert per_600k > per
    assert iht.workspace_bytes(5000, 500_000, 20, 1, iht.MIXED_I8) > one
    L = iht.load()
    for args in ((0, 10, 1, 1, 0), (10, 0, 1, 1, 0), (10, 10, 0, 1, 0), (10, 10, 1, -1, 0), (10, 10, 1, 65, 0)):
        assert L.iht_workspace_bytes(*args) == 0, args
    assert L.iht_workspace_bytes_batch(10, 10, 0, 1, 1, 0) == 0


def test_borrowed_handle_sizes_host_only(lib_path):
    """iht_geno_bytes and iht_stats_bytes size the caller's buffers on the host: the re-tiled matrix
    holds every packed byte (at least ceil(n / 4) p) in 32-subject tiles of 8-byte segments; arguments
    out of range, or a NULL handle, give 0."""
    from paper_1608_01398_amd import iht

    L = iht.load()
    for n, p in ((1, 1), (1000, 5000), (5000, 500_000), (20_000, 2_000_000)):
        b = L.iht_geno_bytes(n, p)
        assert b >= (n + 3) // 4 * p and b % 8 == 0, (n, p, b)
        assert b % (((n + 31) // 32) * 8) == 0  # whole tiles of 8-byte segments per SNP
    assert L.iht_geno_bytes(0, 10) == 0 and L.iht_geno_bytes(10, 0) == 0 and L.iht_geno_bytes(1 << 25, 10) == 0
    assert L.iht_stats_bytes(None) == 0
