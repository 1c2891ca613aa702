"""GPU (HIP C-ABI): the asynchronous registration call, the kernel-timing
calls and the context's workspace accounting.

  * icp_register_async on a side stream writes the same icp_result, bit for
    bit, as the synchronous call on the same inputs, also when consecutive
    calls alternate between two streams.
  * With timing on, one registration records one front-end bracket and one
    launch of each iteration kind per iteration, covering the level pixels of
    every iteration (a single problem in single-pass mode folds the solve
    into pass 2: no solve launches, and the same pose bit for bit as in a
    batch); switching timing on or off clears the totals; the traced (eager)
    launches give the same pose as the untraced ones.
  * The context holds at least the workspace icp_workspace_bytes names for
    the batch it ran.
  * A one-problem registration (which alternates two histograms and window
    predictions between iterations) gives the same pose, bit for bit, after
    stage calls and a batch have used the same context's state.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_1802_03980_amd as icp
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return icp.icp_ctx_create(0)


def upload(p):
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (p.live_depth, p.model_vtx, p.model_nrm))


def test_async_matches_sync(ctx):
    probs = [synth.pair_problem(3), synth.RoomSequence(1, n_frames=2).problem(0)]
    data = [upload(p) for p in probs]
    params = icp.icp_params_default()
    sync = [icp.icp_register(ctx, d, mv, mn, p.K, p.imu_R, p.init_pose, params)
            for p, (d, mv, mn) in zip(probs, data)]
    side = torch.cuda.Stream()
    nbytes = C.sizeof(icp.icp_result)
    outs = [torch.zeros(nbytes, dtype=torch.uint8, device="cuda") for _ in probs]
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for p, (d, mv, mn), out in zip(probs, data, outs):
            icp.icp_register_async(ctx, d, mv, mn, p.K, p.imu_R, p.init_pose, out, params)
    side.synchronize()
    for (Ts, ss), out in zip(sync, outs):
        Ta, sa = icp.result_from_bytes(out.cpu().numpy().tobytes())
        assert np.array_equal(Ta, Ts)
        assert sa["status"] == ss["status"] and sa["iters_total"] == ss["iters_total"]
        for la, ls in zip(sa["levels"], ss["levels"]):
            assert la == ls
    # calls on two streams in turn, with nothing synchronised in between: each
    # call's stream waits for the work the previous call queued, since all
    # calls share the context's workspace
    pairs = [synth.pair_problem(k) for k in (4, 5, 6)]
    pdata = [upload(p) for p in pairs]
    ref = [icp.icp_register(ctx, d, mv, mn, p.K, p.imu_R, p.init_pose, params)[0]
           for p, (d, mv, mn) in zip(pairs, pdata)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs2 = [torch.zeros(nbytes, dtype=torch.uint8, device="cuda") for _ in pairs]
    torch.cuda.synchronize()
    for k, (p, (d, mv, mn), out) in enumerate(zip(pairs, pdata, outs2)):
        with torch.cuda.stream(s1 if k % 2 == 0 else s2):
            icp.icp_register_async(ctx, d, mv, mn, p.K, p.imu_R, p.init_pose, out, params)
    torch.cuda.synchronize()
    for T, out in zip(ref, outs2):
        assert np.array_equal(icp.result_from_bytes(out.cpu().numpy().tobytes())[0], T)
    with pytest.raises(ValueError):  # a result buffer smaller than one icp_result never reaches the library
        icp.icp_register_async(ctx, *data[0], probs[0].K, probs[0].imu_R, probs[0].init_pose, outs[0][:8], params)


def test_batch_async_matches_sync(ctx):
    """icp_register_batch_async queues the batch and returns; two batches
    queued back to back (the second in the reverse order, so a new plan and
    graph are built while the first may still run) give the synchronous
    batch's results bit for bit."""
    probs = [synth.pair_problem(3), synth.pair_problem(4), synth.uneven_problem(6)]
    data = [upload(p) for p in probs]
    items = [dict(live_depth=d, model_vtx=mv, model_nrm=mn, K=p.K, imu_R=p.imu_R, init_pose=p.init_pose)
             for p, (d, mv, mn) in zip(probs, data)]
    params = icp.icp_params_default()
    sync = icp.icp_register_batch(ctx, items, params)
    nbytes = C.sizeof(icp.icp_result) * len(items)
    out1 = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    out2 = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    icp.icp_register_batch_async(ctx, icp.ProblemArray(items), out1, params)
    icp.icp_register_batch_async(ctx, list(reversed(items)), out2, params)
    torch.cuda.synchronize()
    r1 = icp.results_from_bytes(out1.cpu().numpy().tobytes(), len(items), params.levels)
    r2 = icp.results_from_bytes(out2.cpu().numpy().tobytes(), len(items), params.levels)
    for (Ts, ss), (T1, s1), (T2, s2) in zip(sync, r1, reversed(r2)):
        assert np.array_equal(T1, Ts) and s1 == ss
        assert np.array_equal(T2, Ts) and s2 == ss
    with pytest.raises(ValueError):  # a result buffer smaller than the batch never reaches the library
        icp.icp_register_batch_async(ctx, items, out1[:nbytes - 1], params)


def test_kernel_timing_counts_launches(ctx):
    p = synth.RoomSequence(1, n_frames=3).problem(1)
    d, mv, mn = upload(p)
    params = icp.icp_params_default()
    T_graph, _ = icp.icp_register(ctx, d, mv, mn, p.K, p.imu_R, p.init_pose, params)
    icp.icp_ctx_set_timing(ctx, True)
    try:
        T_traced, _ = icp.icp_register(ctx, d, mv, mn, p.K, p.imu_R, p.init_pose, params)
        t = icp.icp_ctx_get_timing(ctx)
    finally:
        icp.icp_ctx_set_timing(ctx, False)
    assert np.array_equal(T_traced, T_graph)
    H, W = p.live_depth.shape
    iters = list(params.iters)[:params.levels]
    level_px = [(W >> l) * (H >> l) for l in range(params.levels)]
    n_it = sum(iters)
    assert t["front_end"]["launches"] == 1 and t["front_end"]["pixels"] == W * H
    for kind in ("pass1", "pass2"):
        assert t[kind]["launches"] == n_it, (kind, t[kind])
        assert t[kind]["total_ms"] > 0.0, kind
    # one problem in single-pass mode: the band kernel, pass 2 and the solve
    # are one launch per iteration (counted as pass 2)
    assert t["band"]["launches"] == 0 and t["solve"]["launches"] == 0
    px_it = sum(i * n for i, n in zip(iters, level_px))
    assert t["pass1"]["pixels"] == px_it and t["pass2"]["pixels"] == px_it
    # a batch of two (and two-pass mode) launches the solve kernel every iteration
    q = synth.RoomSequence(1, n_frames=3).problem(0)
    dq = upload(q)
    items = [dict(live_depth=a, model_vtx=b, model_nrm=c, K=pp.K, imu_R=pp.imu_R, init_pose=pp.init_pose)
             for pp, (a, b, c) in ((p, (d, mv, mn)), (q, dq))]
    icp.icp_ctx_set_timing(ctx, True)
    try:
        batch = icp.icp_register_batch(ctx, items, params)
        icp.icp_register(ctx, d, mv, mn, p.K, p.imu_R, p.init_pose, icp.icp_params_default(pass_mode=1))
        t2 = icp.icp_ctx_get_timing(ctx)
    finally:
        icp.icp_ctx_set_timing(ctx, False)
    assert t2["solve"]["launches"] == 2 * n_it and t2["pass1"]["launches"] == 2 * n_it
    # the batch's solve kernel and the folded solve give the same pose, bit for bit
    assert np.array_equal(batch[0][0], T_graph)
    # switching off cleared the totals, and untraced calls add nothing
    icp.icp_register(ctx, d, mv, mn, p.K, p.imu_R, p.init_pose, params)
    assert all(v["launches"] == 0 and v["total_ms"] == 0.0 for v in icp.icp_ctx_get_timing(ctx).values())


def test_context_workspace_covers_the_batch(ctx):
    probs = [synth.uneven_problem(6), synth.uneven_problem(2)]
    data = [upload(p) for p in probs]
    items = [dict(live_depth=d, model_vtx=mv, model_nrm=mn, K=p.K, imu_R=p.imu_R, init_pose=p.init_pose)
             for p, (d, mv, mn) in zip(probs, data)]
    icp.icp_register_batch(ctx, items, icp.icp_params_default())
    need = icp.icp_workspace_bytes([(p.live_depth.shape[1], p.live_depth.shape[0]) for p in probs])
    assert need > 0 and ctx.workspace_bytes() >= need


def test_state_does_not_leak_between_calls(ctx):
    a = synth.RoomSequence(1, n_frames=3).problem(1)
    b = synth.pair_problem(0)
    da, db = upload(a), upload(b)
    params = icp.icp_params_default()
    T1, s1 = icp.icp_register(ctx, *da, a.K, a.imu_R, a.init_pose, params)
    # stage calls on another problem leave their histogram and prediction behind
    icp.icp_stage_prepare(ctx, *db, b.K, levels=params.levels, params=params)
    for level in range(params.levels):
        T = np.eye(4)
        icp.icp_stage_single_pass(ctx, level, T, 3, 700, 6, params)
    items = [dict(live_depth=d[0], model_vtx=d[1], model_nrm=d[2], K=p.K, imu_R=p.imu_R, init_pose=p.init_pose)
             for p, d in ((a, da), (b, db))]
    batch = icp.icp_register_batch(ctx, items, params)
    T2, s2 = icp.icp_register(ctx, *da, a.K, a.imu_R, a.init_pose, params)
    assert np.array_equal(T1, T2)
    assert s1 == s2
    assert np.array_equal(batch[0][0], T1)  # (the same 1024-pixel tiles alone and in this batch)
