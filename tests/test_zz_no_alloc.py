"""icp_register_noalloc (the registration with no context and no device
allocation, for callers that cannot allocate) against the existing
icp_register_async on the same inputs, through the C ABI: calls in a row on
one GPU share its static array, so each result must be unaffected by what
the previous call left there (a VGA frame, then a smaller 160x120 pair, then
the VGA frame again), bit for bit equal to the context path's, and within
the parity tolerance of the FP64 oracle.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_1802_03980_amd as icp
import synth
from tests.parity_util import assert_registration_matches

pytestmark = pytest.mark.gpu

RES = C.sizeof(icp.icp_result)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _decode(t):
    return icp.result_from_bytes(t.cpu().numpy().tobytes())


def test_noalloc_matches_the_context_path():
    ctx = icp.icp_ctx_create(0)
    params = icp.icp_params_default()
    seq = synth.RoomSequence(0, n_frames=3)
    probs = [seq.problem(0), synth.pair_problem(3), seq.problem(0)]
    first = None
    for k, p in enumerate(probs):
        d, mv, mn = _dev(p.live_depth), _dev(p.model_vtx), _dev(p.model_nrm)
        out_ctx = torch.zeros(RES, dtype=torch.uint8, device="cuda")
        out_static = torch.full((RES,), 0xAB, dtype=torch.uint8, device="cuda")
        icp.icp_register_async(ctx, d, mv, mn, p.K, p.imu_R, p.init_pose, out_ctx, params)
        icp.icp_register_noalloc(d, mv, mn, p.K, p.imu_R, p.init_pose, out_static, params)
        torch.cuda.synchronize()
        assert torch.equal(out_ctx, out_static), (k, p.name)  # every byte of the icp_result
        T, st = _decode(out_static)
        assert_registration_matches(p, params, T, st, f"noalloc call {k} {p.name}")
        if k == 0:
            first = out_static.clone()
        if k == 2:
            assert torch.equal(first, out_static)


def test_noalloc_single_pass_off_and_split_precision():
    """The two-pass and split-precision (MFMA) reductions through the static
    array also equal the context path's."""
    ctx = icp.icp_ctx_create(0)
    p = synth.pair_problem(5)
    d, mv, mn = _dev(p.live_depth), _dev(p.model_vtx), _dev(p.model_nrm)
    for over in (dict(pass_mode=1), dict(reduce_mode=1), dict(converge_window=3, iters=(30, 30, 30))):
        params = icp.icp_params_default(**over)
        a = torch.zeros(RES, dtype=torch.uint8, device="cuda")
        b = torch.zeros(RES, dtype=torch.uint8, device="cuda")
        icp.icp_register_async(ctx, d, mv, mn, p.K, p.imu_R, p.init_pose, a, params)
        icp.icp_register_noalloc(d, mv, mn, p.K, p.imu_R, p.init_pose, b, params)
        torch.cuda.synchronize()
        assert torch.equal(a, b), over


def test_noalloc_rejects_what_does_not_fit():
    """A 1280x720 problem needs 46 MiB of workspace: ICP_ENOMEM before anything
    is queued (the result buffer stays untouched); bad arguments: ICP_EINVAL."""
    big = (720, 1280)
    d = torch.ones(big, dtype=torch.float32, device="cuda")
    m = torch.zeros(big + (3,), dtype=torch.float32, device="cuda")
    out = torch.full((RES,), 7, dtype=torch.uint8, device="cuda")
    K = synth.centred_intrinsics(1280, 720, 787.5)
    assert icp.icp_workspace_bytes([(1280, 720)]) > (32 << 20)
    with pytest.raises(icp.IcpError) as e:
        icp.icp_register_noalloc(d, m, m, K, np.eye(3), np.eye(4), out)
    assert e.value.code == icp.ENOMEM
    with pytest.raises(icp.IcpError) as e:
        icp.icp_register_noalloc(d, m, m, K, np.eye(3) * 1.01, np.eye(4), out)
    assert e.value.code == icp.EINVAL
    with pytest.raises(icp.IcpError) as e:
        icp.icp_register_noalloc(d, m, m, K, np.eye(3), np.eye(4), out, icp.icp_params_default(levels=0))
    assert e.value.code == icp.EINVAL
    torch.cuda.synchronize()
    assert int((out != 7).sum()) == 0
