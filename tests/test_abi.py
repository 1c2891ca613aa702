"""The C-ABI library loads and exports every entry point include/icp.h declares.

CPU-only: no call here touches a GPU (only pure host functions are called).
"""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1802_03980_amd as icp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "icp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(icp_[a-z_]+)\s*\(", src)))


def test_library_built():
    assert os.path.exists(icp.LIB_PATH), "run __graft_entry__.build() first"


def test_exports_match_header():
    declared = _declared()
    assert declared == sorted(icp.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", icp.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (icp_[a-z_]+)\b", out))
    missing = [s for s in declared if s not in exported]
    assert not missing, missing


def test_library_loads_and_host_calls():
    L = icp.lib()
    assert L.icp_abi_version() == icp.ICP_ABI_VERSION
    assert L.icp_strerror(icp.EINVAL) == b"invalid argument"
    p = icp.icp_params_default()
    assert p.levels == 3 and list(p.iters[:3]) == [10, 5, 4]
    assert p.lambda_c == 5.0 and p.use_imu_seed == 1 and p.use_median_filter == 1 and p.anchor_to_imu == 0
    assert abs(p.cos_angle_max - np.cos(np.radians(20))) < 1e-15


def test_struct_sizes_match_header_layout():
    # sizes fixed by natural alignment of the C structs
    assert C.sizeof(icp.icp_intrinsics) == 32
    assert C.sizeof(icp.icp_level_stats) == 40
    assert C.sizeof(icp.icp_stats) == 4 * 40 + 8
    assert C.sizeof(icp.icp_result) == 16 * 8 + C.sizeof(icp.icp_stats)


def test_workspace_bytes_scales_with_pixels():
    vga = icp.icp_workspace_bytes([(640, 480)])
    hd = icp.icp_workspace_bytes([(1280, 720)])
    two = icp.icp_workspace_bytes([(640, 480), (640, 480)])
    # live vertex and normal planes on every level, model maps and depth on
    # the coarser ones (level 0 of those is the caller's buffers)
    assert vga >= 640 * 480 * (24 * (1 + 0.25 + 0.0625) + 28 * (0.25 + 0.0625))
    assert 2.9 < hd / vga < 3.1 and 1.9 < two / vga < 2.1
    assert icp.lib().icp_workspace_bytes(0, None, None, 3) == 0


def test_public_struct_sizes_match_the_c_compiler(tmp_path):
    """Every struct the binding mirrors has the size the C compiler gives it."""
    names = ["icp_intrinsics", "icp_params", "icp_level_stats", "icp_stats", "icp_problem", "icp_result",
             "icp_kernel_time", "icp_server_config", "icp_server_result", "icp_server_counters", "icp_tsdf"]
    src = tmp_path / "sz.c"
    src.write_text("#include <stdio.h>\n#include \"icp.h\"\nint main(void) {\n" +
                   "".join(f'  printf("%zu\\n", sizeof({n}));\n' for n in names) + "  return 0;\n}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    sizes = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    for n, sz in zip(names, sizes):
        assert C.sizeof(getattr(icp, n)) == sz, n


def test_rotations_are_checked_at_the_boundary():
    """The pose is an element of SE(3) (Sec. 3): imu_R, and the initial
    rotation when the IMU seed is off, must be rotations (|R^T R - I| <= 1e-6
    entry by entry, det R > 0); the host-only validation makes the same checks
    as a registration call, so no GPU is needed here."""
    K = (525.0, 525.0, 319.5, 239.5)
    R = np.array([[0.36, 0.48, -0.8], [-0.8, 0.6, 0.0], [0.48, 0.64, 0.6]])  # a rotation
    T = np.eye(4)
    assert icp.icp_validate_problem(640, 480, K, R, T)[0] == icp.OK
    # first-order rounding well inside the tolerance still passes
    assert icp.icp_validate_problem(640, 480, K, R * (1 + 1e-9), T)[0] == icp.OK
    for bad in (R * 1.001, -R, R[[1, 0, 2]], R + np.diag([2e-6, 0, 0]), np.full((3, 3), np.nan)):
        rc, msg = icp.icp_validate_problem(640, 480, K, bad, T)
        assert rc == icp.EINVAL and ("rotation" in msg or "finite" in msg), msg
    # the initial rotation counts only when the IMU seed is off
    Tbad = np.eye(4)
    Tbad[:3, :3] = R * 1.01
    assert icp.icp_validate_problem(640, 480, K, R, Tbad)[0] == icp.OK
    rc, msg = icp.icp_validate_problem(640, 480, K, R, Tbad, icp.icp_params_default(use_imu_seed=0))
    assert rc == icp.EINVAL and "init_pose" in msg
    # the other host checks of a problem
    assert icp.icp_validate_problem(642, 480, K, R, T)[0] == icp.EINVAL  # not divisible by 4
    assert icp.icp_validate_problem(640, 480, (0.0, 525.0, 319.5, 239.5), R, T)[0] == icp.EINVAL
    assert icp.icp_validate_problem(640, 480, K, R, T, icp.icp_params_default(levels=5))[0] == icp.EINVAL


def test_async_results_must_be_device_tensors():
    """The asynchronous calls copy their results device to device: a host
    tensor (or one of another dtype) is refused before the library is called."""
    import torch
    host = torch.zeros(4096, dtype=torch.uint8)
    d = torch.zeros((8, 8), dtype=torch.float32)
    m = torch.zeros((8, 8, 3), dtype=torch.float32)
    with pytest.raises(TypeError, match="result_dev"):
        icp.icp_register_async(None, d, m, m, (1, 1, 1, 1), np.eye(3), np.eye(4), host)
    with pytest.raises(TypeError, match="results_dev"):
        icp.icp_register_batch_async(None, [], host)
