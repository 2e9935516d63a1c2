"""Serving loop through the C ABI.

CPU: argument checks that run before any HIP call.  GPU: a mix of jobs of
several plan classes, sizes and step counts through one server with an
arena too small to admit them all at once; every result must be
bit-identical to sparstencil_run of the same plan alone (each output point's
arithmetic does not depend on which grids share a launch), within its plan's
a-priori bound of the FP64 oracle (and the stated 1e-5 on FP32-state
binary16-split and FP32 jobs), and the job records must be consistent.
"""
import ctypes

import numpy as np
import pytest

import synthetic
from oracle import direct as oracle_direct

from .helpers import STATED_F32, apriori_bound, normwise_err, planes_value

native = pytest.importorskip("paper_2506_22969_amd.native")


def test_server_arguments_rejected_without_device():
    lib = native.lib()
    h = ctypes.c_void_p()
    E = native.SS_E_INVALID
    assert lib.sparstencil_server_create(None, ctypes.c_void_p(256), 1024, 4, 1) == E
    assert lib.sparstencil_server_create(ctypes.byref(h), None, 1024, 4, 1) == E
    assert lib.sparstencil_server_create(ctypes.byref(h), ctypes.c_void_p(256), 0, 4, 1) == E
    assert lib.sparstencil_server_create(ctypes.byref(h), ctypes.c_void_p(256), 1024, 0, 1) == E
    assert lib.sparstencil_server_create(ctypes.byref(h), ctypes.c_void_p(256), 1024, 4, 0) == E
    assert lib.sparstencil_server_create(ctypes.byref(h), ctypes.c_void_p(256), 1024, 4, 17) == E
    jid = ctypes.c_uint64()
    assert lib.sparstencil_submit(None, None, None, None, 1, ctypes.byref(jid)) == E
    assert lib.sparstencil_poll(None, 1, None) == E
    assert lib.sparstencil_job_release(None, 1) == E
    assert lib.sparstencil_server_drain(None) == E
    assert lib.sparstencil_server_destroy(None) == native.SS_OK
    assert lib.sparstencil_server_clock(None) == 0.0


def test_job_info_layout():
    # uint64 + 2 int32 + 2 int64 + 3 doubles
    assert ctypes.sizeof(native.JobInfo) == 8 + 4 + 4 + 8 + 8 + 3 * 8


@pytest.mark.gpu
def test_server_mix_matches_run_alone():
    torch = pytest.importorskip("torch")
    dev = "cuda:0"
    w9, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=(512, 512))
    w9b, _ = synthetic.random_coeffs("box", 1, 2, seed=20, grid_shape=(512, 512))
    assert not np.array_equal(w9, w9b)
    # jobs 1 and 2 are planned apart with equal coefficients: their fused
    # launches batch together, each must still be credited three sweeps
    specs = [  # (coeffs, dims, dtype, engine, boundary, steps[, fused sweeps per launch])
        (w9, (300, 520), "f32_split_f16", "smfmac", "zero", 7),
        (w9, (300, 520), "f32_split_f16", "smfmac", "zero", 11, 3),
        (w9, (300, 520), "f32_split_f16", "smfmac", "zero", 8, 3),
        (w9b, (300, 520), "f32_split_f16", "smfmac", "zero", 10, 3),
        (w9, (130, 264), "f32_split_bf16", "mfma", "zero", 5, 2),
        (w9, (300, 520), "f32_split_f16", "smfmac", "zero", 3),
        (w9, (300, 520), "f32_split_f16", "smfmac", "zero", 12),
        (w9b, (300, 520), "f32_split_f16", "smfmac", "zero", 5),
        (w9, (129, 131), "f32_split_f16", "mfma", "periodic", 4),
        (w9, (256, 1024), "f32_split_bf16", "smfmac", "periodic", 9),
        (w9, (200, 300), "f32", "direct", "zero", 6),
        ("3d", (96, 64, 80), "f32", "direct", "periodic", 3),
        ("3d", (40, 48, 264), "f32_split_f16", "smfmac", "zero", 5),
        ("3d", (24, 48, 264), "f32_split_f16", "smfmac", "zero", 4),
        # two fused 3-D zero-halo jobs of one class: one launch sweeps both
        # grids and computes both bands
        ("3d", (20, 40, 264), "f32_split_f16", "smfmac", "zero", 5, 2),
        ("3d", (12, 56, 132), "f32_split_f16", "smfmac", "zero", 4, 2),
        (w9, (64, 264), "split_bf16", "smfmac", "periodic", 3),
        (w9, (96, 264), "split_bf16", "smfmac", "periodic", 6),
        # planes state on the direct engine: rows of a multiple of 8 values
        # run the LDS-staged kernel, others the plain one; the two plans
        # have equal coefficients but must never share a launch
        (w9, (128, 264), "split_bf16", "direct", "periodic", 4),
        (w9, (128, 262), "split_bf16", "direct", "periodic", 5),
        (w9, (136, 272), "split_bf16", "direct", "zero", 3),
        (w9, (136, 270), "split_bf16", "direct", "zero", 3),
        ("1d", (100003,), "f32_split_f16", "smfmac", "zero", 7, 3),
        ("1d", (77777,), "f32_split_f16", "smfmac", "zero", 9, 3),   # batches with the one above
        ("1d", (4096,), "f32_split_bf16", "mfma", "periodic", 5),
    ]
    plans, jobs, oracle_inputs = [], [], []
    w3 = synthetic.random_coeffs("box", 1, 3, seed=70)[0]
    w1 = synthetic.random_coeffs("box", 1, 1, seed=3, grid_shape=(4096,))[0]
    for i, (w, dims, dtype, engine, bc, steps, *fuse) in enumerate(specs):
        if len(dims) == 3:  # 3-D box of radius 1
            w = w3
        elif len(dims) == 1:
            w = w1
        plan = native.Plan("box", 1, w, dims, dtype, boundary=bc, engine=engine, fuse_steps=fuse[0] if fuse else 1)
        assert plan.info["engine_name"] == engine
        plans.append(plan)
        if dtype == "split_bf16":
            bits = synthetic.grid_bf16_planes(dims, seed=10 + i)
            x0 = torch.from_numpy(bits.view(np.int16)).to(dev)
            start = planes_value(bits)
        else:
            host = synthetic.grid_f32(dims, seed=10 + i)
            x0 = torch.from_numpy(host).to(dev)
            start = host.astype(np.float64)
        jobs.append((plan, x0, steps))
        oracle_inputs.append((w, start, dtype, bc == "periodic"))

    # reference: each job alone through sparstencil_run
    refs = []
    for plan, x0, steps in jobs:
        a = x0.clone()
        b = torch.empty_like(a)
        plan.run(a, b, steps, torch.cuda.current_stream().cuda_stream)
        refs.append(b)
    torch.cuda.synchronize()

    # arena for the largest job and half as much again: the rest must queue
    largest = max(p.grid_bytes for p, _, _ in jobs)
    arena_bytes = 3 * ((largest + 255) // 256 * 256)
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
    outs = [torch.full_like(x0, -1) for _, x0, _ in jobs]
    with native.Server(arena, arena_bytes, max_jobs=64, num_streams=3) as srv:
        ids = [srv.submit(plan, x0, out, steps) for (plan, x0, steps), out in zip(jobs, outs)]
        srv.drain()
        infos = []
        for jid, (plan, x0, steps) in zip(ids, jobs):
            st, info = srv.poll(jid)
            assert st == native.SS_OK, info
            assert info["state"] == 2 and info["status"] == 0
            assert info["steps_done"] == info["steps_total"] == steps
            assert info["t_submit"] <= info["t_admit"] <= info["t_done"] <= srv.clock()
            infos.append(info)
            srv.release(jid)
            with pytest.raises(native.SparStencilError):
                srv.poll(jid)
        # the arena cannot hold every job at once, so some were admitted late
        assert max(i["t_admit"] for i in infos) > min(i["t_done"] for i in infos)
    torch.cuda.synchronize()
    for i, (out, ref) in enumerate(zip(outs, refs)):
        assert torch.equal(out, ref), f"job {i} differs from the job run alone"
    # and every served result against the FP64 oracle
    for i, ((plan, _x0, steps), out, (w, start, dtype, periodic)) in enumerate(zip(jobs, outs, oracle_inputs)):
        host = out.cpu().numpy()
        got = planes_value(host.view(np.uint16)) if dtype == "split_bf16" else host.astype(np.float64)
        ref = oracle_direct.run(start, w, steps, periodic=periodic)
        err = normwise_err(got, ref)
        kk = len(plan.table(native.Q_KERNEL_PERM)) if plan.info["engine_name"] != "direct" else 0
        tol = apriori_bound(plan.info, w, steps, dtype, kk)
        print(f"job {i} {plan.info['engine_name']} {dtype} {start.shape} err={err:.3e} tol={tol:.3e}")
        assert err <= tol, f"job {i}"
        if dtype in ("f32_split_f16", "f32"):
            assert err <= STATED_F32, f"job {i}"
    for p in plans:
        p.close()


@pytest.mark.gpu
def test_server_rejects_job_larger_than_arena():
    torch = pytest.importorskip("torch")
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=(64, 64))
    arena = torch.empty(4096, dtype=torch.uint8, device="cuda:0")
    with native.Plan("box", 1, w, (64, 64), "f32_split_f16") as plan, \
            native.Server(arena, 4096, max_jobs=2, num_streams=1) as srv:
        x = torch.zeros(64, 64, device="cuda:0")
        y = torch.empty_like(x)
        with pytest.raises(native.SparStencilError) as e:
            srv.submit(plan, x, y, 3)
        assert e.value.status == native.SS_E_NOMEM
        with pytest.raises(native.SparStencilError) as e:
            srv.submit(plan, x, y, 0)
        assert e.value.status == native.SS_E_INVALID
