"""Benchmark: quadruped environment steps per second on one MI355X.

One bench "step" = one full rollout of the workload batch: 4096 quadruped
environments x 1000 environment steps (dt 0.05 s, 10 substeps), seeded
synthetic reset perturbations and actions, inputs resident in HBM before the
timed region. `value` is the fused forward rate (env-steps/s). The plain
per-phase path and the forward+VJP rate are reported beside it, plus the
roofline of the dominant kernel and the FP64 oracle timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import gc
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

from paper_2106_13281_amd import braxmi, synth  # noqa: E402

# the other legs tune their launch shape on the first steps of their own
# rollout (brax_autotune_on), so that the trials see the contacts of use
TUNE_STEPS = 200
PEAK_FP32_TFLOPS = 157.3    # published FP32 vector peak: 256 CU x 2.4 GHz x 256 FLOP/clock (packed FP32 FMA)
ISSUE_FP32_TFLOPS = 78.6     # the same without packed FP32 (not generated: disabled at build)
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_flops(name, key="mean"):
    """Oracle-counted FLOP per environment step: the forward ("mean") or one
    reverse sweep ("vjp_mean")."""
    with open(os.path.join(ROOT, "tests", "golden", "algorithmic_flops.json")) as f:
        return json.load(f)["workloads"][name][key]


# the sources k_fused is compiled from (its translation unit and the headers it includes)
KERNEL_SOURCES = ("bx_kernels.hip", "bx_phys.h", "bx_access.h", "bx_tables.h", "bx_internal.h", "bx_pair.h",
                  "bx_pair_lanes.h", "bx_pair_adj.h", "bx_adj.h")


def measured_traffic():
    """HBM bytes per k_fused launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a 256 MiB copy), or None
    when the kernel sources differ from the ones the counters were taken on."""
    path = os.path.join(ROOT, "profiles", "k_fused_quadruped_4096x1000_counters.md")
    try:
        with open(path) as f:
            text = f.read()
        want = re.search(r"kernel_source_sha256: ([0-9a-f]{64})", text).group(1)
        nbytes = int(re.search(r"hbm_bytes_per_launch: (\d+)", text).group(1))
    except (OSError, AttributeError):
        return None
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2106_13281_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return nbytes if h.hexdigest() == want else None


def plain_bytes_per_env_substep(system, t=0):
    """Bytes the plain per-phase kernels read and write per environment and
    substep (FP32; 13 floats of state per body): kinematic 2x13 per body; joint
    2x13 state + one action per axis + a 12-float slot per joint; contact 13
    state + a 7-float slot per candidate; potential 2x13 state per body + the
    6-float child or parent half of every joint's slot; collision 2x13 state
    per body + every candidate's slot. = 312 nb + 200 nj + 4 D + 108 nc."""
    nb, nj, nd, nc = system.n_bodies[t], system.n_joints[t], system.n_dof[t], system.n_contacts[t]
    return 312 * nb + 200 * nj + 4 * nd + 108 * nc


def make_inputs(system, wl, seed=0):
    E = system.n_envs
    ang, root = synth.reset_noise(seed, E, system.d_max, wl.angle_noise, wl.root_noise)
    angles = system.default_angles(0)[:, None] + torch.from_numpy(np.ascontiguousarray(ang.T))
    s0 = system.default_qp(angles.contiguous().cuda(), torch.from_numpy(np.ascontiguousarray(root.T)).cuda())
    acts = torch.from_numpy(synth.acts_to_device_layout(synth.actions(seed, wl.steps, E, system.a_max,
                                                                      wl.act_range))).cuda()
    torch.cuda.synchronize()
    return s0, acts


def time_calls(fn, reps, warmup):
    """Average ms per call with HIP events on torch's current stream (the one the library uses).
    Python's cyclic garbage collector is held off over the timed calls (as timeit does): a full
    collection inside a loop of short calls stalls the host for tens of milliseconds."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    try:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
    finally:
        gc.enable()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(s0, acts, system, budget_s=4.0, budget_1core_s=1.5, reps=3):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload (all environments, as many leading steps as fit the budget), and
    on one core on a smaller sample; built -O3 -march=native on this host,
    each figure the median of `reps` timed runs."""
    import oracle
    build_cmd = oracle.use_native()
    o = oracle.Oracle(synth.system_text("quadruped"))
    E = system.n_envs
    X = synth.from_soa(*(t.cpu().numpy() for t in s0.fields()), n_body=o.nb)
    A = acts.cpu().numpy().transpose(0, 2, 1)[:, :, :o.na].astype(np.float64)   # [T][E][A]
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    o.rollout(X, A[:2], threads=threads)
    per = (time.perf_counter() - t0) / (2 * E)          # seconds per env-step on all threads
    T = int(max(2, min(A.shape[0], budget_s / max(per * E, 1e-9))))

    def median_time(fn):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), ts

    dt, ts = median_time(lambda: o.rollout(X, A[:T], threads=threads))
    model = oracle.cpu_model()
    full = {"value": E * T / dt, "unit": "env-steps/s", "cores": threads, "kind": "oracle",
            "cpu": model, "build": build_cmd,
            "sample": f"all {E} quadruped environments x first {T} of the {A.shape[0]} steps, FP64, "
                      f"OpenMP over environments on {threads} threads of {model}; median of {reps} runs "
                      f"({', '.join(f'{x:.2f}' for x in ts)} s)"}
    n1 = min(E, 256)
    T1 = int(max(2, min(A.shape[0], budget_1core_s / max(per * threads * n1, 1e-9))))
    dt1, ts1 = median_time(lambda: o.rollout(X[:n1], A[:T1, :n1], threads=1))
    one = {"value": n1 * T1 / dt1, "unit": "env-steps/s", "cores": 1, "kind": "oracle", "cpu": model,
           "sample": f"{n1} of the {E} quadruped environments x first {T1} steps, FP64, one thread; median of "
                     f"{reps} runs ({', '.join(f'{x:.2f}' for x in ts1)} s)"}
    return full, one


def segment_adjoint(n):
    """The adjoint of one 10-step checkpoint segment of the differentiation
    workload (1024 quadrupeds) from its tape (brax_rollout_vjp_tape), n times."""
    wd = synth.WORKLOADS["quadruped_diff"]
    dsys = braxmi.System(synth.system_text("quadruped"), wd.envs, device=0)
    d0, dall = make_inputs(dsys, wd)
    K = 10
    acts = dall[:K].contiguous()
    tape = torch.empty((K, dsys.tape_step_floats), dtype=torch.float32, device="cuda")
    dsys.rollout_tape(d0, acts, tape=tape)
    g = dsys.new_state()
    for f in g.fields():
        f.normal_()
    gi = dsys.new_state()
    gA = torch.empty((K, dsys.a_max, dsys.n_envs), dtype=torch.float32, device="cuda")
    ms = time_calls(lambda: dsys.rollout_vjp_tape(tape, acts, g, g_in=gi, g_acts=gA), max(n, 1), 0)
    log(f"segment adjoint: {ms * 1e3:.1f} us per {wd.envs}x{K} segment ({max(n, 1)} calls)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=100, help="env steps timed for the plain path")
    # the headline batch runs at a fixed launch shape, so that every run (and
    # every profiler pass) times the same launch: 4 environments per
    # wavefront and one wavefront per block give 1024 wavefronts, one per
    # SIMD; the autotuner's other candidates for this batch time within about
    # 2% of it, and it picks among them by run-to-run noise
    ap.add_argument("--schedule", default="4,1",
                    help="fused launch shape 'ENVS_PER_WAVE,WAVES_PER_BLOCK' for the quadruped batch, or 'auto'")
    ap.add_argument("--only", choices=["all", "fused", "segment_adjoint"], default="all",
                    help="fused: time only the fused forward rollout (for profiler runs), after a 256 MiB "
                         "device copy that calibrates the HBM byte counters; segment_adjoint: only the "
                         "adjoint of one 10-step checkpoint segment of the differentiation workload from "
                         "its tape, --steps times without warm-up (for profiler runs; the kernel trace gives "
                         "its duration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the environments are independent and need no exchange); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    if args.only == "segment_adjoint":
        segment_adjoint(args.steps)
        return

    wl = synth.WORKLOADS["quadruped"]
    E, T = wl.envs, wl.steps
    system = braxmi.System(synth.system_text("quadruped"), E, device=0)
    s0, acts = make_inputs(system, wl)
    out = system.new_state()
    log(f"inputs ready: {E} envs x {T} steps")
    if args.schedule == "auto":
        epw, wpb = system.autotune_on(s0, acts[:TUNE_STEPS])
    else:
        epw, wpb = system.set_schedule(*(int(x) for x in args.schedule.split(",")))
    log(f"schedule ({args.schedule}): {epw} envs/wave, {wpb} waves/block")

    if args.only == "fused":
        # a plain copy of known size (256 MiB read + 256 MiB written) next to the
        # kernel, to scale the profiler's FETCH_SIZE / WRITE_SIZE readings
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        flush = torch.empty(160 << 20, dtype=torch.float32, device="cuda")
        flush.fill_(2.0)          # 640 MiB written: evicts the 256 MiB last-level cache
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst, flush

    # fused forward: the timed region is K full rollouts
    ms_fused = time_calls(lambda: system.rollout(s0, acts, out=out), args.steps, args.warmup)
    fused = E * T / (ms_fused / 1e3)
    log(f"fused forward: {ms_fused:.2f} ms per rollout, {fused:.3e} env-steps/s")
    if args.only == "fused":
        print(json.dumps({"fused_fwd_env_steps_per_s": fused, "ms_per_rollout": ms_fused}), flush=True)
        return

    # plain per-phase path (one launch per phase per substep), shorter horizon
    Tp = min(args.plain_steps, T)
    ms_plain = time_calls(lambda: system.rollout(s0, acts[:Tp], out=out, flags=braxmi.BRAX_PLAIN), 1, 1)
    plain = E * Tp / (ms_plain / 1e3)
    ms_plain_g = time_calls(lambda: system.rollout(s0, acts[:Tp], out=out, flags=braxmi.BRAX_PLAIN | braxmi.BRAX_GRAPH),
                            1, 1)
    plain_g = E * Tp / (ms_plain_g / 1e3)
    S = system.substeps[0]
    plain_launches = 5 * S * Tp            # kinematic, joint, contact, potential, collision per substep
    plain_bytes = plain_bytes_per_env_substep(system) * E * S * Tp
    log(f"plain forward: {ms_plain:.2f} ms per {Tp}-step rollout, {plain:.3e} env-steps/s; "
        f"graph-replayed {ms_plain_g:.2f} ms; {plain_bytes / (ms_plain / 1e3) / 1e9:.0f} GB/s")

    # environment layer after the step (reward, termination, auto-reset,
    # observation), single steps graph-replayed, ant-like parameters
    system.env_configure([dict(root=0, forward_weight=1.0, healthy_reward=1.0, ctrl_cost=0.5, z_min=0.2, z_max=1.0)])
    est = system.new_state()
    for x, y in zip(est.fields(), s0.fields()):
        x.copy_(y)
    eobs = torch.empty(system.obs_dim, E, device="cuda")
    erew = torch.empty(E, device="cuda")
    edone = torch.empty(E, dtype=torch.uint8, device="cuda")
    n_env_steps = 100
    eact = acts[0].clone()      # the policy's action buffer (fixed address, as a replayed graph wants)

    def env_loop():
        for _ in range(n_env_steps):
            system.env_step(est, eact, s0, out=est, obs=eobs, reward=erew, done=edone, flags=braxmi.BRAX_GRAPH)
    ms_env = time_calls(env_loop, 1, 1)
    env_rate = E * n_env_steps / (ms_env / 1e3)
    log(f"environment step: {ms_env / n_env_steps * 1e3:.1f} us per step of {E} environments")

    # forward + VJP: the differentiation workload (1024 quadrupeds x 100 steps),
    # gradient of a loss w.r.t. all actions; the whole forward tape is kept in
    # device memory (rollout_grad's default where it fits), and the same with
    # checkpoints every 10 steps (each segment's tape recomputed)
    wd = synth.WORKLOADS["quadruped_diff"]
    dsys = braxmi.System(synth.system_text("quadruped"), wd.envs, device=0)
    d0, dacts = make_inputs(dsys, wd)
    k_vjp = braxmi.checkpoint_interval(dsys, wd.steps)

    def fwd_bwd(k):
        A = dacts.detach().clone().requires_grad_(True)
        out_d = braxmi.rollout_grad(dsys, d0, A, k=k)
        loss = -(out_d.pos[0, 0] - d0.pos[0, 0]).sum() + 1e-3 * (A ** 2).sum()
        loss.backward()
        return A.grad
    ms_vjp = time_calls(lambda: fwd_bwd(k_vjp), 5, 2)
    fwd_vjp = wd.envs * wd.steps / (ms_vjp / 1e3)
    ms_vjp10 = time_calls(lambda: fwd_bwd(10), 5, 2)
    tape_mb = wd.steps * dsys.tape_step_floats * 4 / 1e6
    log(f"forward+VJP: {ms_vjp:.2f} ms per {wd.envs}x{wd.steps} rollout gradient, {fwd_vjp:.3e} env-steps/s "
        f"(tape of {k_vjp} steps, {tape_mb:.0f} MB); checkpoints every 10 steps {ms_vjp10:.2f} ms")

    # the other workloads: biped forward; mixed batch (one persistent launch
    # over 8192 environments of four system types), direct and graph-replayed,
    # forward and forward+VJP
    extra = {}
    wb = synth.WORKLOADS["biped"]
    bsys = braxmi.System(synth.system_text("biped"), wb.envs, device=0)
    b0, bacts = make_inputs(bsys, wb)
    bsys.autotune_on(b0, bacts[:TUNE_STEPS])
    bout = bsys.new_state()
    ms_b = time_calls(lambda: bsys.rollout(b0, bacts, out=bout), args.steps, args.warmup)
    extra["biped_fwd_env_steps_per_s"] = wb.envs * wb.steps / (ms_b / 1e3)
    extra["biped_fwd_frac"] = algorithmic_flops("biped") * wb.envs * wb.steps / (ms_b / 1e3) / 1e12 / PEAK_FP32_TFLOPS
    log(f"biped forward: {ms_b:.2f} ms per {wb.envs}x{wb.steps} rollout")
    # the quadruped at twice the environments: 8192 fill every SIMD with
    # wavefronts (4096 leave the GPU one wavefront per SIMD at most)
    E2 = 2 * E
    qsys = braxmi.System(synth.system_text("quadruped"), E2, device=0)
    q0, qacts = make_inputs(qsys, wl)
    qsys.autotune_on(q0, qacts[:TUNE_STEPS])
    qout = qsys.new_state()
    ms_q = time_calls(lambda: qsys.rollout(q0, qacts, out=qout), args.steps, args.warmup)
    extra["quadruped_8192_fwd_env_steps_per_s"] = E2 * T / (ms_q / 1e3)
    extra["quadruped_8192_fwd_frac"] = algorithmic_flops("quadruped") * E2 * T / (ms_q / 1e3) / 1e12 / PEAK_FP32_TFLOPS
    log(f"quadruped {E2} forward: {ms_q:.2f} ms per {E2}x{T} rollout")
    del qsys, q0, qacts, qout
    # planar runner with target-angle actuators
    wc = synth.WORKLOADS["cheetah"]
    csys = braxmi.System(synth.system_text("cheetah"), wc.envs, device=0)
    c0, cacts = make_inputs(csys, wc)
    csys.autotune_on(c0, cacts[:TUNE_STEPS])
    cout = csys.new_state()
    ms_c = time_calls(lambda: csys.rollout(c0, cacts, out=cout), args.steps, args.warmup)
    extra["cheetah_fwd_env_steps_per_s"] = wc.envs * wc.steps / (ms_c / 1e3)
    extra["cheetah_fwd_frac"] = algorithmic_flops("cheetah") * wc.envs * wc.steps / (ms_c / 1e3) / 1e12 / PEAK_FP32_TFLOPS
    log(f"cheetah forward: {ms_c:.2f} ms per {wc.envs}x{wc.steps} rollout")
    # grasp: the manipulator with finger-box body-body contacts
    wg = synth.WORKLOADS["grasp"]
    gsys = braxmi.System(synth.system_text("grasp"), wg.envs, device=0)
    g0, gacts = make_inputs(gsys, wg)
    gsys.autotune_on(g0, gacts[:TUNE_STEPS])
    gout = gsys.new_state()
    ms_g = time_calls(lambda: gsys.rollout(g0, gacts, out=gout), args.steps, args.warmup)
    extra["grasp_fwd_env_steps_per_s"] = wg.envs * wg.steps / (ms_g / 1e3)
    extra["grasp_fwd_frac"] = algorithmic_flops("grasp") * wg.envs * wg.steps / (ms_g / 1e3) / 1e12 / PEAK_FP32_TFLOPS
    extra["grasp_workload"] = (f"manipulator with six finger-box body-body candidates (each finger capsule's two ends "
                               f"and axis segment), box within reach, "
                               f"{wg.envs} environments x {wg.steps} steps, actions U(-1,1)")
    log(f"grasp forward: {ms_g:.2f} ms per {wg.envs}x{wg.steps} rollout")

    types = synth.mixed_assignment(0)
    msys = braxmi.System([synth.system_text(n) for n in synth.MIXED_TYPES], len(types), env_desc=types, device=0)
    m0 = msys.default_qp(None, None)
    Tm = 1000
    macts = torch.from_numpy(synth.acts_to_device_layout(
        synth.actions(0, Tm, len(types), msys.a_max, 1.0))).cuda()
    msys.autotune_on(m0, macts[:TUNE_STEPS])
    mout = msys.new_state()
    ms_m = time_calls(lambda: msys.rollout(m0, macts, out=mout), args.steps, args.warmup)
    ms_mg = time_calls(lambda: msys.rollout(m0, macts, out=mout, flags=braxmi.BRAX_GRAPH), args.steps,
                       args.warmup)
    extra["mixed_fwd_env_steps_per_s"] = len(types) * Tm / (ms_m / 1e3)
    mixed_flop = sum(algorithmic_flops(n) * int((types == t).sum()) for t, n in enumerate(synth.MIXED_TYPES)) * Tm
    extra["mixed_fwd_frac"] = mixed_flop / (ms_m / 1e3) / 1e12 / PEAK_FP32_TFLOPS
    extra["mixed_fwd_graph_env_steps_per_s"] = len(types) * Tm / (ms_mg / 1e3)
    # single steps, launched one by one vs replayed from a captured graph
    ms_ms = time_calls(lambda: msys.step(m0, macts[0], out=mout), 50, 5)
    ms_msg = time_calls(lambda: msys.step(m0, macts[0], out=mout, flags=braxmi.BRAX_GRAPH), 50, 5)
    extra["mixed_step_us"] = ms_ms * 1e3
    extra["mixed_step_graph_us"] = ms_msg * 1e3
    Tv = 100

    def mixed_fwd_bwd():
        A = macts[:Tv].detach().clone().requires_grad_(True)
        o2 = braxmi.rollout_grad(msys, m0, A)
        (o2.pos.sum() + 1e-3 * (A ** 2).sum()).backward()
        return A.grad
    ms_mv = time_calls(mixed_fwd_bwd, 3, 1)
    extra["mixed_fwd_vjp_env_steps_per_s"] = len(types) * Tv / (ms_mv / 1e3)
    extra["mixed_workload"] = ("8192 environments: 2048 chains, 3277 quadrupeds, 2048 bipeds, 819 manipulators "
                               "(seeded permutation), reset pose, actions U(-1,1); forward 1000 steps, "
                               f"forward+VJP 100 steps (checkpoint interval "
                               f"{braxmi.checkpoint_interval(msys, Tv)} steps: the whole tape where it fits)")
    log(f"mixed forward: {ms_m:.2f} ms ({ms_mg:.2f} ms graph); step {ms_ms * 1e3:.1f} us "
        f"({ms_msg * 1e3:.1f} us graph); forward+VJP {ms_mv:.2f} ms")

    fpe = algorithmic_flops("quadruped")
    vpe = algorithmic_flops("quadruped", "vjp_mean")
    achieved = fpe * E * T / (ms_fused / 1e3) / 1e12
    result = {
        "metric": "quadruped env-steps/s, fwd and fwd+VJP, fused vs plain kernels, 1 MI355X",
        "value": fused,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_fused,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"quadruped rollout: {E} environments x {T} steps, dt 0.05 s, 10 substeps, "
                               f"actions U(-1,1), seed 0", "envs": E, "env_steps": T, "substeps": 10,
                   "schedule": {"envs_per_wave": epw, "waves_per_block": wpb}},
        "fused_fwd_env_steps_per_s": fused,
        "plain_fwd_env_steps_per_s": plain,
        "fused_over_plain": fused / plain,
        "plain_fwd_graph_env_steps_per_s": plain_g,
        "env_step_env_steps_per_s": env_rate,
        "env_step_workload": f"quadruped {E} environments, single environment steps (step, reward, termination, "
                             f"auto-reset, observation) graph-replayed, {n_env_steps} steps",
        "fwd_vjp_env_steps_per_s": fwd_vjp,
        "fwd_vjp_frac": fwd_vjp * (fpe + vpe) / 1e12 / PEAK_FP32_TFLOPS,
        "fwd_vjp_flop_per_env_step": fpe + vpe,
        "fwd_vjp_workload": f"quadruped {wd.envs} environments x {wd.steps} steps, the whole forward tape "
                            f"({tape_mb:.0f} MB) kept in device memory; algorithmic work per env-step = forward "
                            f"{fpe:.0f} + one reverse sweep {vpe:.0f} FLOP",
        "fwd_vjp_ckpt10_env_steps_per_s": wd.envs * wd.steps / (ms_vjp10 / 1e3),
        "plain_fwd_gbs": plain_bytes / (ms_plain / 1e3) / 1e9,
        "plain_bytes_per_env_substep": plain_bytes_per_env_substep(system),
        "plain_us_per_launch": ms_plain * 1e3 / plain_launches,
        "plain_graph_us_per_launch": ms_plain_g * 1e3 / plain_launches,
        **extra,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(),
                     "kernel": "k_fused", "flop_per_env_step": fpe,
                     "peak_note": "published FP32 vector peak (packed FP32 FMA); packed FP32 is disabled at "
                                  f"build, so the reachable issue rate is {ISSUE_FP32_TFLOPS} TFLOP/s: frac vs it = "
                                  f"{achieved / ISSUE_FP32_TFLOPS:.4f}"},
    }
    if not args.no_cpu:
        result["cpu_baseline"], result["cpu_baseline_1core"] = cpu_baseline(s0, acts, system)
        log(f"cpu baseline: {result['cpu_baseline']}; one core: {result['cpu_baseline_1core']}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
