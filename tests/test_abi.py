"""CPU-side checks of the C-ABI library: it loads, exports every function that
include/cfog.h declares, rejects invalid arguments before touching a device,
and its register DFT codelets are exact against a naive DFT (host build).
No compute runs here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfog.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", txt, flags=re.M)) - {"if"})


@pytest.fixture(scope="module")
def lib():
    from paper_1808_06194_amd import cfog
    if not os.path.exists(cfog.LIB_PATH):
        from paper_1808_06194_amd import build
        build.build()
    return cfog.load()


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("cfog_extract", "match_batch", "cfog_ctx_create", "match_batch_workspace_size"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1808_06194_amd import cfog
    names = _declared()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(cfog.EXPORTS) == set(names)


def test_status_strings(lib):
    from paper_1808_06194_amd import cfog
    assert cfog.status_str(0) == "ok"
    assert "invalid" in cfog.status_str(cfog.CFOG_EINVAL)
    assert cfog.status_str(12345) == "unknown status"


def test_null_context_is_rejected(lib):
    from paper_1808_06194_amd import cfog
    assert lib.cfog_extract(None, None, 8, 8, 8, 9, 0.8, -1, None, None, None, 0, None) == cfog.CFOG_EINVAL
    assert lib.match_batch(None, None, 0, 9, 1, None, 0, None) == cfog.CFOG_EINVAL
    assert lib.match_batch_workspace_size(None, None, 0, 9, 1) == ctypes.c_size_t(-1).value
    assert lib.cfog_ctx_create(0, None) == cfog.CFOG_EINVAL
    assert lib.cfog_ctx_destroy(None) == 0
    assert lib.match_batch_noalloc(None, None, 0, 9, 1, None) == cfog.CFOG_EINVAL
    assert lib.cfog_noalloc_scratch_bytes() == 48 << 20


def test_job_struct_layout_matches_header():
    from paper_1808_06194_amd import cfog
    assert ctypes.sizeof(cfog.cfog_job) == 96
    assert cfog.cfog_job.out.offset == 72 and cfog.cfog_job.surfaces.offset == 80
    assert cfog.cfog_job.subpix.offset == 88


def test_image_struct_layout_matches_header():
    from paper_1808_06194_amd import cfog
    assert ctypes.sizeof(cfog.cfog_image) == 40
    assert cfog.cfog_image.row_stride.offset == 8 and cfog.cfog_image.H.offset == 16
    assert cfog.cfog_image.d_vol.offset == 24 and cfog.cfog_image.d_sat.offset == 32


def test_extract_batch_workspace_and_argument_checks(lib):
    """The batch workspace is the per-image workspaces of the images with a
    SAT, each rounded up to 256 bytes; invalid batches are rejected on the
    host."""
    from paper_1808_06194_amd import cfog
    shapes = [(37, 53), (1, 1), (2048, 2048), (129, 7)]
    one = [lib.cfog_extract_workspace_size(H, W) for H, W in shapes]
    assert one[2] == max(8 * (2048 * 16 + 128 * 2048), 8 * (2048 * 32 + 64 * 2048))
    assert one[3] == max(8 * (129 * 1 + 9 * 7), 8 * (129 * 1 + 5 * 7))
    assert cfog.extract_batch_workspace_size(shapes) == sum((b + 255) // 256 * 256 for b in one)
    assert cfog.extract_batch_workspace_size(shapes, with_sat=False) == 0
    assert cfog.extract_batch_workspace_size([]) == 0
    assert lib.cfog_extract_batch_workspace_size(None, 3) == 0
    arr = (cfog.cfog_image * 1)()
    assert lib.cfog_extract_batch(None, arr, 1, 9, 0.8, -1, 2, None, 0, None) == cfog.CFOG_EINVAL


def test_max_window(lib):
    assert lib.cfog_max_window() >= 192


def test_fft_size_choice(lib):
    from paper_1808_06194_amd import cfog
    assert cfog.fft_size(100, 20) >= 140 and cfog.fft_size(48, 10) >= 68
    assert cfog.fft_size(128, 32) >= 192 and cfog.fft_size(300, 10) == 0
    assert lib.cfog_set_plan(None, 10, 2, 16) == cfog.CFOG_EINVAL


def test_dft_codelets_host_build(tmp_path):
    src = os.path.join(ROOT, "tests", "cpp", "dft_codelets.cpp")
    exe = tmp_path / "dft_codelets"
    inc = os.path.join(ROOT, "paper_1808_06194_amd", "csrc")
    r = subprocess.run(["/opt/rocm/bin/hipcc", "-std=c++17", "-O2", "-x", "hip", "--offload-arch=gfx950",
                        "-I", inc, src, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout


def test_server_structs_match_header():
    from paper_1808_06194_amd import cfog
    assert ctypes.sizeof(cfog.cfog_server_config) == 40
    assert cfog.cfog_server_config.max_batch_surf.offset == 32
    assert ctypes.sizeof(cfog.cfog_request_info) == 56
    assert cfog.cfog_request_info.batch_reqs.offset == 48
    assert ctypes.sizeof(cfog.cfog_server_stats) == 80


def test_reject_result_layout():
    from paper_1808_06194_amd import cfog
    assert ctypes.sizeof(cfog.cfog_reject_result) == 216
    assert cfog.cfog_reject_result.rmse.offset == 192 and cfog.cfog_reject_result.status.offset == 208


def test_server_null_handles_are_rejected(lib):
    from paper_1808_06194_amd import cfog
    i32, i64 = ctypes.c_int32(), ctypes.c_int64()
    assert lib.cfog_server_create(0, None, None) == cfog.CFOG_EINVAL
    assert lib.cfog_server_destroy(None) == cfog.CFOG_OK
    assert lib.cfog_server_add_pair(None, None, 8, 8, 8, None, 8, 8, 8, ctypes.byref(i32)) == cfog.CFOG_EINVAL
    assert lib.cfog_server_submit(None, 0, None, 1, 8, 1, None, None, ctypes.byref(i64)) == cfog.CFOG_EINVAL
    assert lib.cfog_server_poll(None, None, 0, 0, ctypes.byref(i32)) == cfog.CFOG_EINVAL
    assert lib.cfog_server_get_stats(None, None) == cfog.CFOG_EINVAL


def test_server_scheduler_simulation(tmp_path):
    """The serving scheduler (admission by memory, FIFO continuous batching,
    LRU eviction) driven by a simulated executor, built for the host."""
    src = os.path.join(ROOT, "tests", "cpp", "sched_sim.cpp")
    exe = tmp_path / "sched_sim"
    inc = os.path.join(ROOT, "paper_1808_06194_amd", "csrc")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-I", inc, src,
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-2000:]
    assert "ALL OK" in r.stdout


def test_channel_split_planner(tmp_path):
    """The host-side choice of the matcher's last-round channel split
    (split_plan.hpp), built for the host with the sanitizers."""
    src = os.path.join(ROOT, "tests", "cpp", "split_plan_test.cpp")
    exe = tmp_path / "split_plan_test"
    inc = os.path.join(ROOT, "paper_1808_06194_amd", "csrc")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-I", inc, src,
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-2000:]
    assert "ALL OK" in r.stdout


def test_window_rule_host_build(tmp_path):
    """The control-point window rule the kernels and the server share
    (window.hpp), built for the host with the sanitizers: control points at
    INT_MIN / INT_MAX, +-N/2 and +-r around every edge, flush boxes and one
    past them, against a 128-bit reference and pixel enumeration."""
    src = os.path.join(ROOT, "tests", "cpp", "window_test.cpp")
    exe = tmp_path / "window_test"
    inc = os.path.join(ROOT, "paper_1808_06194_amd", "csrc")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-I", inc, src, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-2000:]
    assert "ALL OK" in r.stdout
