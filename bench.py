#!/usr/bin/env python3
"""MO-PCG throughput on one MI355X.

Workload (the headline configuration): -Lap u + u = f, P2 MO-FEM on the
x-normal domain {0 < X < 1, 0 < Y < 1 + 0.3 sin(pi X)}, homogeneous
Dirichlet, n = 2049 nodes per direction (q = 2047 unknowns per direction),
f = manufactured source + N(0, 1e-3^2) noise (seed 1234 + b), a batch of 16
independent instances, MO-PCG with the spectral single-term preconditioner
to a relative FP64 residual of 1e-8.

One step = the whole hot path over the batch: the full-node load
M3 F M (eq. (74)) and the batched MO-PCG solve (operator apply, spectral
preconditioner, FP64 recurrence, true-residual check).  The one-off setup
(1D assembly and the two FP64 eigen-decompositions) runs before timing and
is reported separately.

value = mixed-path solves/s (by default the forward transforms in BF16 and the
back transforms in split BF16 on MFMA, flexible PCG, FP64 recurrence and
residual); the FP64 path (FP64 MFMA transforms) is timed on the same GPU and
reported beside it.  Kernel times come from the library's HIP-event
tracing, recorded on the launch stream inside the timed region.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
F64_PEAK_TFLOPS = 78.6
I8_PEAK_TOPS = 5000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(F0, k, m, gamma, tol, U_gpu0):
    """The oracle (NumPy/SciPy FP64) on one instance of the same workload."""
    import numpy as np

    from oracle.problems import XNormalProblem
    from oracle.solvers import SpectralPrec, mo_pcg
    from workloads import L_profile, dL_profile
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # threadpoolctl missing: report the host's logical CPUs
        threads = os.cpu_count()
    P = XNormalProblem(k, m, "dirichlet", L_profile, dL_profile, gamma=gamma)
    S = SpectralPrec(*P.prec_pairs("sylv-matched"))   # the library's elliptic pencils
    R = P.rhs(F0)
    t0 = time.perf_counter()
    U, info = mo_pcg(P.apply, S.apply, R, tol=tol, maxit=200)
    dt = time.perf_counter() - t0
    fwd = float(np.linalg.norm(U_gpu0 - U) / np.linalg.norm(U))
    back = float(np.linalg.norm(R - P.apply(U_gpu0)) / np.linalg.norm(R))
    return dict(value=1.0 / dt, unit="solves/s", cores=int(threads), kind="oracle",
                sample="1 of the 16 instances (item 0, seed 1234), FP64 MO-PCG to rel 1e-8, "
                       "eigen-setup excluded; %d iterations in %.1f s" % (info["iters"], dt)), fwd, back


# HBM traffic of the transform GEMM, from two rocprofv3 --pmc passes over
# "bench.py --steps 1 --warmup 0 --no-cpu-baseline --fp64-steps 0 --int8-steps 0 --heat-steps 0 --dib-steps 0
# --adjoint 0 --imex-steps 0 --uneven 0 --paper-prec 0" (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch, averaged over that kernel's dispatches),
# each scaled by the ratio true bytes / counter reading of a plain 512 MiB
# copy ("bench.py --copy-calibration").  The figures hold for the kernel
# source they were taken on: if k_gemm.hip or device_common.h (its tile
# order) changes, traffic is reported null.
TRAFFIC = {
    # mixed mode -> (sha256 of k_gemm.hip + device_common.h, (q, batch), bytes per launch)
    "bf16fwdvs": ("6cc5159f7964d1cd36946228fa206c9343bd0ef25742071d2eb2c447c3fd0029", (2047, 16), 1.780e9),
}
FETCH_SCALE = 2.000   # 512 MiB copy: true bytes / FETCH_SIZE reading
WRITE_SCALE = 1.000   # 512 MiB copy: true bytes / WRITE_SIZE reading


def measured_traffic(mode, q, batch):
    import hashlib
    rec = TRAFFIC.get(mode)
    if rec is None:
        return None
    h = hashlib.sha256()
    for name in ("k_gemm.hip", "device_common.h"):
        with open(os.path.join(ROOT, "paper_2109_01173_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    sha = h.hexdigest()
    if sha != rec[0] or tuple(rec[1]) != (q, batch):
        return None
    return rec[2]


def copy_calibration(torch):
    """A plain device copy of known size, for scaling byte counters."""
    n = 512 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 5}), flush=True)


def uneven_leg(mf, torch, np, n_inst, prec, prec_name, rds_steps=100):
    """Uneven mixed batch: n_inst instances; seed 5 draws n from {257, 513,
    1025, 2049}, then k from 1..4, then the type: elliptic (P_k x-normal,
    Dirichlet, gamma = 1, manufactured f + 1e-3 noise, rel 1e-8, the mixed
    path's transforms) or reaction-diffusion (DIB on the rectangle [0,20]^2,
    Neumann, lumped P1 for k = 1 and P_k otherwise, tau = 1e-2, rds_steps IMEX
    steps of both species at rel 1e-10, FP64 transforms).  Same-shape
    instances of one type form one batched group.  The elliptic groups are
    solved one after another (pcg_solve) and together on four streams
    (pcg_solve_many); the reaction-diffusion groups step one after another.
    The elliptic groups are also solved grouped by shape (pcg_solve_many
    with grouped=True: one batched solve per shape class, all element orders
    in the same launches), and the reaction-diffusion groups are also
    replayed from one HIP graph per group on their own streams; the
    whole-job time takes the faster form of each part.  The groups' set-up
    (assembly, eigen-decompositions) runs on a pool of host threads."""
    from paper_2109_01173_amd.problems import Rect, XNormal
    from workloads import dib_initial, dib_params, elliptic_batch
    rng = np.random.default_rng(5)
    ns = rng.choice([257, 513, 1025, 2049], size=n_inst)
    ks = rng.integers(1, 5, size=n_inst)
    types = rng.integers(0, 2, size=n_inst)  # 0 elliptic, 1 reaction-diffusion
    shapes = {}
    for n, k, ty in zip(ns.tolist(), ks.tolist(), types.tolist()):
        shapes[(ty, n, k)] = shapes.get((ty, n, k), 0) + 1
    t0 = time.perf_counter()
    p = dib_params()
    kin = [p["rho"], p["A1"], p["A2"], p["B"], p["C"], p["D"], p["alpha"], p["gamma"], p["k2"], p["k3"]]

    def build(item):
        # one shape group: assembly, eigen-decompositions and upload in the
        # library (its calls release the interpreter, so groups build in parallel)
        gi, ((ty, n, k), cnt) = item
        m = int(round((n - 1) / k))
        if ty == 0:
            G = XNormal(k, m, "dirichlet", gamma=1.0, precision=prec)
            F = torch.from_numpy(elliptic_batch(G.n, 1.0, cnt, sigma=1e-3, seed0=5000 + 100 * gi)).cuda()
            rhs = G.rhs_op.apply(F)
            torch.cuda.synchronize()
            return 0, dict(op=G.op, prec=G.prec, rhs=rhs, U=torch.empty_like(rhs), tol=1e-8, maxit=300,
                           flags=mf.PCG_FLEXIBLE | mf.PCG_ZERO_GUESS, _keep=G,
                           workspace=mf.pcg_workspace(G.op, G.prec, cnt))
        lumped = k == 1
        # split-BF16 transforms: three flexible PCG iterations per solve to rel
        # 1e-10 cost less than one with FP64 transforms
        G = Rect(k, m, "neumann", length=20.0, lumped=lumped, imex=True, closed_form=lumped,
                 precision=mf.PREC_BF16X3)
        init = [dib_initial(G.q, seed=7000 + 100 * gi + j) for j in range(cnt)]
        # species-major state: eta of every item, then theta of every item
        st0 = torch.from_numpy(np.stack([e for e, _ in init] + [t for _, t in init])).cuda()
        stepper = mf.Imex(G.op, G.prec, G.mass, 1e-2, [1.0, p["d_theta"]], kinetics=mf.KIN_DIB, kin=kin,
                          tol=1e-10, maxit=50, flags=mf.PCG_FLEXIBLE)
        r = dict(G=G, st0=st0, st=st0.clone(), stepper=stepper, batch=cnt, ws=stepper.workspace(cnt))
        torch.cuda.synchronize()
        return 1, r

    # four set-ups at a time with a quarter of the host threads each, largest
    # first (one set-up's threads synchronise at every reduction step, so
    # running more than the cores allow would stall them all)
    from concurrent.futures import ThreadPoolExecutor
    workers = 4
    items = list(enumerate(sorted(shapes.items())))
    items.sort(key=lambda it: -it[1][0][1])
    prev = mf.set_host_threads(max(1, mf.set_host_threads(0) // workers))
    try:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            built = list(ex.map(build, items))
    finally:
        mf.set_host_threads(prev)
    groups = [g for ty, g in built if ty == 0]
    rds = [r for ty, r in built if ty == 1]
    setup = time.perf_counter() - t0
    n_ell = sum(int(g["rhs"].shape[0]) for g in groups)
    n_rds = sum(r["batch"] for r in rds)
    for g in groups:  # warm-up (also the kernels' first use)
        mf.pcg_solve(g["op"], g["prec"], g["rhs"], g["U"], tol=1e-8, maxit=300, flags=g["flags"],
                     workspace=g["workspace"])
    for r in rds:
        r["stepper"].step(r["st"], r["batch"], workspace=r["ws"])
        r["st"].copy_(r["st0"])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for g in groups:
        mf.pcg_solve(g["op"], g["prec"], g["rhs"], g["U"], tol=1e-8, maxit=300, flags=g["flags"],
                     workspace=g["workspace"])
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t
    streams = [torch.cuda.Stream() for _ in range(4)]
    t = time.perf_counter()
    outs, status = mf.pcg_solve_many(groups, [streams[i % 4] for i in range(len(groups))])
    torch.cuda.synchronize()
    dt_many = time.perf_counter() - t
    its = np.concatenate([o[0] for o in outs]) if outs else np.zeros(1)
    # grouped: one batched solve per shape class (one launch per stage over its
    # instances of every k), each class on its own stream
    shape_of = sorted({int(g["rhs"].shape[1]) for g in groups})
    cstreams = [torch.cuda.Stream() for _ in shape_of]   # one stream per shape class
    gstreams = [cstreams[shape_of.index(int(g["rhs"].shape[1]))] for g in groups]
    mf.pcg_solve_many(groups, gstreams, grouped=True)   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    outs_g, status_g = mf.pcg_solve_many(groups, gstreams, grouped=True)
    torch.cuda.synchronize()
    dt_grp = time.perf_counter() - t
    its_g = np.concatenate([o[0] for o in outs_g]) if outs_g else np.zeros(1)
    # each shape class alone (where the grouped time goes)
    class_ms = {}
    for q_c in shape_of:
        idx = [i for i, g in enumerate(groups) if int(g["rhs"].shape[1]) == q_c]
        torch.cuda.synchronize()
        t = time.perf_counter()
        mf.pcg_solve_many([groups[i] for i in idx], [streams[0]] * len(idx), grouped=True)
        torch.cuda.synchronize()
        class_ms[str(q_c)] = [sum(int(groups[i]["rhs"].shape[0]) for i in idx),
                              round((time.perf_counter() - t) * 1e3, 2)]
    rds_its = []
    t = time.perf_counter()
    for r in rds:
        for _ in range(rds_steps):
            rds_its.append(int(r["stepper"].step(r["st"], r["batch"], workspace=r["ws"]).max()))
    torch.cuda.synchronize()
    dt_rds = time.perf_counter() - t
    finite = all(bool(torch.isfinite(r["st"]).all()) for r in rds)
    eager_final = [r["st"].clone() for r in rds]
    # the same steps replayed from one HIP graph per group (as many PCG
    # iterations budgeted per solve as the eager steps needed: the DIB solves
    # converge in one), the groups on their own streams
    for r in rds:
        r["st"].copy_(r["st0"])
        r["graph"] = mf.ImexGraph(r["stepper"], r["st"], r["batch"], iters_per_step=max(rds_its))
        r["side"] = torch.cuda.Stream()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for r in rds:
        with torch.cuda.stream(r["side"]):
            r["graph"].launch(rds_steps)
    torch.cuda.synchronize()
    dt_rds_g = time.perf_counter() - t
    g_ok = True
    for r, ref in zip(rds, eager_final):
        its_g_r, st_g_r, _ = r["graph"].result(raise_on_error=False)
        d = float((r["st"] - ref).norm() / ref.norm())
        g_ok = g_ok and bool((st_g_r == 0).all()) and d <= 1e-12
        rds_its.append(int(its_g_r.max()))
    finite = finite and all(bool(torch.isfinite(r["st"]).all()) for r in rds)
    job = dt_grp + min(dt_rds, dt_rds_g)
    log("uneven batch: %d instances (%d elliptic in %d groups, %d shapes, %d reaction-diffusion in %d groups): "
        "elliptic %.1f solves/s one group at a time, %.1f groups on streams, %.1f grouped by shape; "
        "reaction-diffusion %.1f instance-steps/s (%d steps each) eager, %.1f replayed from graphs on streams "
        "(graph states %s the eager ones to 1e-12); whole job %.2f s = %.1f instances/s"
        % (n_inst, n_ell, len(groups), len(shape_of), n_rds, len(rds), n_ell / dt_seq, n_ell / dt_many,
           n_ell / dt_grp, n_rds * rds_steps / dt_rds if dt_rds > 0 else 0.0, rds_steps,
           n_rds * rds_steps / dt_rds_g if dt_rds_g > 0 else 0.0, "equal to" if g_ok else "DIFFER FROM",
           job, n_inst / job))
    return {"uneven_batch": {"workload": "%d instances, n in {257,513,1025,2049}, k in 1..4, type in {elliptic, "
                                         "reaction-diffusion} (seed 5); elliptic: P_k x-normal, Dirichlet, gamma=1, "
                                         "rel 1e-8, %s transforms; reaction-diffusion: DIB rectangle [0,20]^2, "
                                         "Neumann, tau=1e-2, %d steps, rel 1e-10, bf16x3 transforms, flexible PCG"
                                         % (n_inst, prec_name, rds_steps),
                             "elliptic_instances": n_ell, "elliptic_groups": len(groups),
                             "solves_per_s_sequential": round(n_ell / dt_seq, 2),
                             "solves_per_s_streams": round(n_ell / dt_many, 2), "streams": 4,
                             "solves_per_s_grouped": round(n_ell / dt_grp, 2), "shape_classes": len(shape_of),
                             "class_items_ms": class_ms,
                             "iterations_max": int(max(its.max(), its_g.max())),
                             "status_ok": all(st == 0 for st in status + status_g),
                             "rds_instances": n_rds, "rds_groups": len(rds),
                             "rds_instance_steps_per_s": round(n_rds * rds_steps / dt_rds, 2) if dt_rds > 0 else None,
                             "rds_instance_steps_per_s_graphs": round(n_rds * rds_steps / dt_rds_g, 2)
                             if dt_rds_g > 0 else None, "rds_graph_states_equal_eager": g_ok,
                             "rds_iterations_max": max(rds_its) if rds_its else 0, "rds_finite": finite,
                             "job_s": round(job, 3), "instances_per_s": round(n_inst / job, 2),
                             "setup_s": round(setup, 2)}}


def radial_spectrum_peak(np, U):
    """Dominant radial wavenumber bin of a field on a uniform square grid (FFT
    power of the mean-free field, summed over rings of unit width) - a
    rounding-insensitive summary of a Turing pattern."""
    F = np.abs(np.fft.rfft2(U - U.mean())) ** 2
    n = U.shape[0]
    kx = np.fft.fftfreq(n)[:, None] * n
    ky = np.fft.rfftfreq(U.shape[1])[None, :] * U.shape[1]
    rb = np.rint(np.sqrt(kx ** 2 + ky ** 2)).astype(int)
    spec = np.bincount(rb.ravel(), F.ravel())
    return int(spec[1:].argmax() + 1)


HEAT_PREC = {"f32": "PREC_F32", "bf16x3": "PREC_BF16X3", "bf16fwdvs": "PREC_BF16_FWD_VS"}


def heat_leg(mf, torch, np, nsteps, eager_steps, prec_name="f32"):
    """Heat equation (eqs. (89)-(96)): P4 on the x-normal domain, Neumann,
    n = 2049, d = 0.1, tau = 1e-3, U0 ~ U[0,1) (seed 42), f = 0; transforms
    in prec_name (f32: FP32 operands and accumulation; bf16x3: split BF16;
    bf16fwdvs: plain BF16 forward, S rounded to BF16, last back transform
    split) with the FP64 residual and recurrence, flexible PCG to rel 1e-10
    per step.  `eager_steps` steps
    through mofem_imex_step (they also fix the graph's iteration budget),
    then `nsteps` steps replayed from the captured HIP graph."""
    from paper_2109_01173_amd.problems import XNormal
    from workloads import heat_initial
    t0 = time.perf_counter()
    G = XNormal(4, 512, "neumann", gamma=0.0, imex=True, precision=getattr(mf, HEAT_PREC[prec_name]))
    setup = time.perf_counter() - t0
    st = torch.from_numpy(heat_initial(G.q, seed=42)[None]).cuda()
    mk = lambda: mf.Imex(G.op, G.prec, G.mass, 1e-3, [0.1], tol=1e-10, maxit=200, flags=mf.PCG_FLEXIBLE)
    stepper = mk()
    ws = stepper.workspace(1)
    mass0 = float(G.mass.apply(st).sum())
    torch.cuda.synchronize()
    t = time.perf_counter()
    its = [int(stepper.step(st, 1, workspace=ws)[0]) for _ in range(eager_steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    # the rough initial data need the most iterations in the first steps (35
    # falling to 14 over the ten eager steps); the budget covers the later
    # eager steps with two to spare, and a replayed step that ran out of it
    # would show in the graph's status
    budget = max(its[len(its) // 2:]) + 2
    g = mf.ImexGraph(mk(), st, 1, iters_per_step=budget)
    torch.cuda.synchronize()
    t = time.perf_counter()
    g.launch(nsteps)
    torch.cuda.synchronize()
    dtg = time.perf_counter() - t
    gi, gst, grr = g.result(raise_on_error=False)
    mass1 = float(G.mass.apply(st).sum())
    out = {"imex_heat_p4": {
        "workload": "heat P4 x-normal, Neumann, n=2049, d=0.1, tau=1e-3, U0 ~ U[0,1) seed 42, %s transforms, "
                    "FP64 residual, rel 1e-10 per step, %d graph-replayed steps after %d eager steps"
                    % (prec_name, nsteps, eager_steps),
        "graph_steps_per_s": round(nsteps / dtg, 3), "steps": nsteps, "graph_iteration_budget": budget,
        "graph_max_iterations": int(gi.max()), "graph_status_ok": bool(np.all(gst == 0)),
        "last_step_relres": float(np.max(grr)),
        "eager_steps_per_s": round(eager_steps / dt, 3), "eager_iterations_per_step": round(float(np.mean(its)), 2),
        "eager_iterations": its,
        "transforms": prec_name, "setup_s": round(setup, 2),
        "mass_drift_rel": abs(mass1 - mass0) / abs(mass0),
        "time_reached": round(1e-3 * (nsteps + eager_steps), 4)}}
    log("heat P4 (%s transforms): %.1f steps/s replayed (%d steps, budget %d, max %d iterations), %.1f eager; "
        "mass drift %.2e" % (prec_name, nsteps / dtg, nsteps, budget, gi.max(), eager_steps / dt,
                             abs(mass1 - mass0) / abs(mass0)))
    del g
    return out


def dib_leg(mf, torch, np, nsteps):
    """Two-species reaction-diffusion (Sec. 7, eqs. (98)-(103)): DIB kinetics on
    the rectangle [0,20]^2, Neumann, n = 1025 (lumped P1 with m = 1024 and P2
    with m = 512), d_theta / d_eta = 20, tau = 1e-2, equilibrium + U[-1e-3,
    1e-3) (seed 7), rectangle preconditioner (exact in FP64) with split-BF16
    transforms and the flexible PCG at rel 1e-10 per step (three iterations
    per solve cost less than one with FP64 transforms); `nsteps` steps (10^4:
    T = 100) replayed from a HIP graph, plus the Turing pattern's statistics
    at the end."""
    from paper_2109_01173_amd.problems import Rect
    from workloads import dib_initial, dib_params
    p = dib_params()
    kin = [p["rho"], p["A1"], p["A2"], p["B"], p["C"], p["D"], p["alpha"], p["gamma"], p["k2"], p["k3"]]
    out = {}
    for key, k, m, lumped in (("imex_dib_p1", 1, 1024, True), ("imex_dib_p2", 2, 512, False)):
        t0 = time.perf_counter()
        G = Rect(k, m, "neumann", length=20.0, lumped=lumped, imex=True, closed_form=lumped,
                 precision=mf.PREC_BF16X3)
        setup = time.perf_counter() - t0
        eta, theta = dib_initial(G.q, seed=7)
        st = torch.from_numpy(np.stack([eta, theta])).cuda()
        mk = lambda: mf.Imex(G.op, G.prec, G.mass, 1e-2, [1.0, p["d_theta"]], kinetics=mf.KIN_DIB, kin=kin,
                             tol=1e-10, maxit=50, flags=mf.PCG_FLEXIBLE)
        stepper = mk()
        ws = stepper.workspace(1)
        warm = 10
        torch.cuda.synchronize()
        t = time.perf_counter()
        its = [int(stepper.step(st, 1, workspace=ws).max()) for _ in range(warm)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        # as many iterations as the eager steps needed (the last one confirms
        # convergence on the true residual inside the replay); a step needing
        # more would show in the graph's status
        g = mf.ImexGraph(mk(), st, 1, iters_per_step=max(its))
        torch.cuda.synchronize()
        t = time.perf_counter()
        g.launch(nsteps - warm)
        torch.cuda.synchronize()
        dtg = time.perf_counter() - t
        gi, gst, _ = g.result(raise_on_error=False)
        e, th = st.cpu().numpy()
        name = "lumped P1" if lumped else "P2"
        out[key] = {"workload": "DIB %s rectangle [0,20]^2, Neumann, n=1025, tau=1e-2, two species, bf16x3 transforms, rel 1e-10 per "
                                "step, T=%g (%d steps: %d eager, the rest replayed from a HIP graph)"
                                % (name, 1e-2 * nsteps, nsteps, warm),
                    "graph_steps_per_s": round((nsteps - warm) / dtg, 2), "steps": nsteps,
                    "eager_steps_per_s": round(warm / dt, 2), "iterations_per_step": max(its),
                    "graph_max_iterations": int(gi.max()), "graph_status_ok": bool(np.all(gst == 0)),
                    "transforms": "bf16x3", "eigenbasis": "closed form" if lumped else "dense eigen-solve",
                    "setup_s": round(setup, 2),
                    "final_state": {"eta_mean": float(e.mean()), "eta_var": float(e.var()),
                                    "theta_mean": float(th.mean()), "theta_var": float(th.var()),
                                    "eta_peak_radial_bin": radial_spectrum_peak(np, e), "finite": bool(
                                        np.isfinite(e).all() and np.isfinite(th).all())}}
        log("DIB %s: %.1f steps/s replayed (%d steps to T = %g); eta mean %.3e var %.3e, peak bin %d"
            % (name, (nsteps - warm) / dtg, nsteps, 1e-2 * nsteps, e.mean(), e.var(), radial_spectrum_peak(np, e)))
        del g, G, st, stepper, ws
    return out


# relative residual of every solve in the gradient leg: above the FP64
# evaluation floor of the n = 257 operators (measured 1.1e-12 for the P2
# x-normal operator, 2.5e-14 for the lumped P1 IMEX operator)
TOL_ADJ = 1e-11


def adjoint_leg(mf, torch, np, nsteps=100, checkpoint=50):
    """Gradients through the solver (torch.autograd over the library's
    adjoint): (1) a reaction-diffusion instance of the uneven draw's kind (DIB,
    lumped P1 on [0,20]^2, n = 257, 100 steps, checkpoint every 50),
    J = ||eta(T) - eta_t||^2 + ||theta(T) - theta_t||^2 with seeded targets,
    dJ/d(d_eta) and dJ/d(d_theta); (2) an elliptic instance (P2 x-normal,
    n = 257, batch 4), J = ||U - U_t||^2, dJ/dF along a seeded direction;
    each against central finite differences of the GPU forward map."""
    from paper_2109_01173_amd.autograd import EllipticSolve, ImexRollout
    from paper_2109_01173_amd.problems import Rect, XNormal
    from workloads import dib_initial, dib_params, elliptic_batch
    p = dib_params()
    kin = [p["rho"], p["A1"], p["A2"], p["B"], p["C"], p["D"], p["alpha"], p["gamma"], p["k2"], p["k3"]]
    tau = 1e-2
    G = Rect(1, 256, "neumann", length=20.0, lumped=True, imex=True, closed_form=True)
    eta0, theta0 = dib_initial(G.q, seed=11)
    rng = np.random.default_rng(12)
    target = torch.from_numpy(np.stack([1e-3 * rng.standard_normal((G.q, G.q)),
                                        0.5 + 1e-3 * rng.standard_normal((G.q, G.q))])).cuda()
    s0 = torch.from_numpy(np.stack([eta0, theta0])).cuda()
    d0 = [1.0, p["d_theta"]]

    def rollout(dvec, grad):
        d = torch.tensor(dvec, dtype=torch.float64, device="cuda", requires_grad=grad)
        out = ImexRollout.apply(s0, d, G, tau, nsteps, mf.KIN_DIB, kin, TOL_ADJ, 50, 0, checkpoint)
        return d, ((out - target) ** 2).sum()
    torch.cuda.synchronize()
    t = time.perf_counter()
    d, J = rollout(d0, True)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t
    t = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t
    g = d.grad.cpu().numpy()
    fd_err = []
    for i in range(2):
        h = 1e-5 * d0[i]
        with torch.no_grad():
            jp = float(rollout([d0[j] + (h if j == i else 0.0) for j in range(2)], False)[1])
            jm = float(rollout([d0[j] - (h if j == i else 0.0) for j in range(2)], False)[1])
        fd = (jp - jm) / (2 * h)
        fd_err.append(abs(fd - g[i]) / abs(fd))
    # elliptic: dJ/dF along a direction
    Ge = XNormal(2, 128, "dirichlet", gamma=1.0)
    F = elliptic_batch(Ge.n, 1.0, 4, sigma=1e-3, seed0=77)
    Ut = torch.from_numpy(np.random.default_rng(13).standard_normal((4, Ge.q, Ge.q)) * 1e-2).cuda()
    Ft = torch.from_numpy(F).cuda().requires_grad_(True)
    gam = torch.tensor(1.0, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    U = EllipticSolve.apply(Ft, gam, Ge, TOL_ADJ, 300, 0)
    Je = ((U - Ut) ** 2).sum()
    Je.backward()
    torch.cuda.synchronize()
    t_ell = time.perf_counter() - t
    E = np.random.default_rng(14).standard_normal(F.shape)
    h = 1e-3
    with torch.no_grad():
        jp = float(((EllipticSolve.apply(torch.from_numpy(F + h * E).cuda(), gam, Ge, TOL_ADJ, 300, 0) - Ut) ** 2).sum())
        jm = float(((EllipticSolve.apply(torch.from_numpy(F - h * E).cuda(), gam, Ge, TOL_ADJ, 300, 0) - Ut) ** 2).sum())
    fd = (jp - jm) / (2 * h)
    ell_err = abs(fd - float((Ft.grad.cpu().numpy() * E).sum())) / abs(fd)
    log("adjoint: DIB n=257 %d steps (checkpoint %d) forward %.2f s backward %.2f s, FD rel err d_eta %.1e "
        "d_theta %.1e; elliptic P2 n=257 batch 4 dJ/dF FD rel err %.1e (%.2f s)"
        % (nsteps, checkpoint, t_fwd, t_bwd, fd_err[0], fd_err[1], ell_err, t_ell))
    return {"adjoint": {"workload": "DIB lumped P1 rectangle [0,20]^2, Neumann, n=257, tau=1e-2, %d steps, "
                                    "checkpoint every %d, J = ||state(T) - target||^2, gradient in (d_eta, "
                                    "d_theta); elliptic P2 x-normal n=257 batch 4, J = ||U - U_t||^2, gradient "
                                    "in F" % (nsteps, checkpoint),
                        "rollout_forward_s": round(t_fwd, 3), "rollout_backward_s": round(t_bwd, 3),
                        "grad_d": [float(x) for x in g],
                        "fd_rel_err_d_eta": float(fd_err[0]), "fd_rel_err_d_theta": float(fd_err[1]),
                        "elliptic_forward_backward_s": round(t_ell, 3), "fd_rel_err_dF": float(ell_err)}}


def paper_prec_leg(mf, torch, np, G_head, batch, nsteps):
    """The paper's own product preconditioners, applied by banded Cholesky
    solves, beside the spectral one: (1) the banded apply on the headline
    shape (HBM-bound: each of its two launches reads the input and its
    scratch and writes both, 32 B per entry); (2) eq. (80) on a smaller
    elliptic P2 case (its iteration count grows with q; the spectral count
    does not); (3) heat steps (P4, n = 2049) preconditioned by eq. (95)."""
    from paper_2109_01173_amd.problems import XNormal
    from workloads import heat_initial
    out = {}
    q = G_head.q
    prec = G_head.product_prec()
    R = torch.randn(batch, q, q, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    Z = torch.empty_like(R)
    ws = torch.empty(prec.workspace_size(batch), dtype=torch.uint8, device="cuda")
    prec.apply(R, Z, workspace=ws)
    torch.cuda.synchronize()
    mf.trace_select((mf.TRACE_BCHOL,))
    mf.trace_enable(True)
    for _ in range(5):
        prec.apply(R, Z, workspace=ws)
    torch.cuda.synchronize()
    mf.trace_enable(False)
    mf.trace_select(None)
    c_ms, c_n, c_items = mf.trace_read(mf.TRACE_BCHOL)
    gbs = 32.0 * q * q * c_items / (c_ms * 1e-3) / 1e9 if c_ms > 0 else 0.0
    out["banded_apply"] = {"workload": "eq. (80) B1^-1 R (A+B2)^-1, P2 q=%d, batch %d" % (q, batch),
                           "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(gbs / HBM_PEAK_GBS, 4), "avg_launch_ms": round(c_ms / max(c_n, 1), 4),
                           "apply_ms": round(2 * c_ms / max(c_n, 1), 4)}
    del R, Z, ws, prec
    # elliptic eq. (80) vs spectral (FP64 both) at q = 255
    G = XNormal(2, 128, "dirichlet", gamma=1.0)
    from workloads import elliptic_batch
    F = torch.from_numpy(elliptic_batch(G.n, 1.0, batch, sigma=1e-3, seed0=1234)).cuda()
    rhs = G.rhs_op.apply(F)
    U = torch.empty_like(rhs)
    res = {}
    for name, pr in (("eq80", G.product_prec()), ("spectral", G.prec)):
        mf.pcg_solve(G.op, pr, rhs, U, tol=1e-8, maxit=20000, flags=mf.PCG_ZERO_GUESS)
        torch.cuda.synchronize()
        t = time.perf_counter()
        its, rr, _ = mf.pcg_solve(G.op, pr, rhs, U, tol=1e-8, maxit=20000, flags=mf.PCG_ZERO_GUESS)
        torch.cuda.synchronize()
        res[name] = (batch / (time.perf_counter() - t), int(its.max()))
    out["paper_eq80_elliptic"] = {"workload": "elliptic P2 x-normal, n=257 (q=255), Dirichlet, gamma=1, batch %d, "
                                              "rel 1e-8, FP64" % batch,
                                  "solves_per_s": round(res["eq80"][0], 2), "iterations": res["eq80"][1],
                                  "spectral_solves_per_s": round(res["spectral"][0], 2),
                                  "spectral_iterations": res["spectral"][1]}
    log("paper eq. (80) at q=255: %d iterations, %.1f solves/s (spectral: %d iterations, %.1f solves/s)"
        % (res["eq80"][1], res["eq80"][0], res["spectral"][1], res["spectral"][0]))
    del G, F, rhs, U
    # heat with eq. (95) against the spectral preconditioner, both with the
    # stopping rule of Sec. 6 (||R_s|| <= tau ||R_0||), FP64
    tau, d = 1e-3, 0.1
    G = XNormal(4, 512, "neumann", gamma=0.0, imex=True)
    U0 = torch.from_numpy(heat_initial(G.q, seed=42)[None]).cuda()
    res = {}
    for name, pr in (("eq95", G.product_prec(scales=(d * tau,))), ("spectral", G.prec)):
        st = U0.clone()
        stepper = mf.Imex(G.op, pr, G.mass, tau, [d], tol=tau, maxit=5000, flags=mf.PCG_TAU_STOP)
        ws = stepper.workspace(1)
        stepper.step(st, 1, workspace=ws)
        torch.cuda.synchronize()
        t = time.perf_counter()
        its = [int(stepper.step(st, 1, workspace=ws)[0]) for _ in range(nsteps)]
        torch.cuda.synchronize()
        res[name] = (nsteps / (time.perf_counter() - t), float(np.mean(its)))
    out["paper_eq95_heat_p4"] = {"workload": "heat P4 x-normal, Neumann, n=2049, d=0.1, tau=1e-3, stop at "
                                             "||R_s|| <= tau ||R_0|| (Sec. 6), FP64",
                                 "steps_per_s": round(res["eq95"][0], 3),
                                 "iterations_per_step": round(res["eq95"][1], 2),
                                 "spectral_steps_per_s": round(res["spectral"][0], 3),
                                 "spectral_iterations_per_step": round(res["spectral"][1], 2)}
    log("paper eq. (95) heat P4, tau stop: %.2f steps/s, %.1f iterations/step (spectral FP64: %.2f steps/s, "
        "%.1f iterations/step)" % (res["eq95"][0], res["eq95"][1], res["spectral"][0], res["spectral"][1]))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--int8-steps", type=int, default=1,
                    help="timed steps of the FP64-accurate path with INT8 digit-product transforms (0 skips it)")
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--n", type=int, default=2049)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--mixed", default="bf16fwdvs", choices=["bf16x2", "bf16x3", "bf16", "bf16fwd", "bf16fwdvs"],
                    help="transform precision of the mixed path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--heat-steps", type=int, default=1000,
                    help="graph-replayed steps of the heat P4 leg (0 skips it)")
    ap.add_argument("--heat-prec", default="f32,bf16fwdvs",
                    help="comma list of transform precisions of the heat P4 leg (%s); the first is the "
                         "configured one, the others are reported beside it" % ", ".join(sorted(HEAT_PREC)))
    ap.add_argument("--dib-steps", type=int, default=10000,
                    help="steps of each DIB leg (10^4 reaches T = 100; 0 skips them)")
    ap.add_argument("--adjoint", type=int, default=1, help="run the gradient leg (0 skips it)")
    ap.add_argument("--imex-steps", type=int, default=10,
                    help="eager steps of the heat leg and of the product-preconditioner heat leg")
    ap.add_argument("--uneven", type=int, default=64,
                    help="instances of the uneven-batch leg (0 skips it)")
    ap.add_argument("--paper-prec", type=int, default=1,
                    help="run the leg of the paper's product preconditioners (eqs. (80), (95)); 0 skips it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    bad = [hp for hp in args.heat_prec.split(",") if hp not in HEAT_PREC]
    if bad:
        ap.error("--heat-prec: unknown precision(s) %s" % ", ".join(bad))
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build runs every instance batch on a single "
              "MI355X; a multi-GPU run is not provided (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        copy_calibration(torch)
        return

    from paper_2109_01173_amd import mofem as mf
    from paper_2109_01173_amd.problems import XNormal
    from workloads import elliptic_batch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    k, gamma = 2, 1.0
    m = (args.n - 1) // k
    B = args.batch

    t0 = time.perf_counter()
    mixed = {"bf16x2": (mf.PREC_BF16X2, mf.TRACE_GEMM_BF16X2, 2, "gemm_bf16_kernel<BF_X2A|BF_X2B,*>"),
             "bf16x3": (mf.PREC_BF16X3, mf.TRACE_GEMM_BF16X3, 3, "gemm_bf16_kernel<BF_X3,*>"),
             "bf16": (mf.PREC_BF16, mf.TRACE_GEMM_BF16, 1, "gemm_bf16_kernel<BF_HH,*>"),
             # forward transforms one BF16 product, back transforms split: the
             # roofline is taken on the split (dominant) back-transform kernel
             "bf16fwd": (mf.PREC_BF16_FWD, mf.TRACE_GEMM_BF16X3, 3, "gemm_bf16_kernel<BF_X3,*>"),
             # as bf16fwd, the first back transform splitting V_s only (S in BF16)
             "bf16fwdvs": (mf.PREC_BF16_FWD_VS, mf.TRACE_GEMM_BF16X3, 3, "gemm_bf16_kernel<BF_X3,*>")}[args.mixed]
    G = XNormal(k, m, "dirichlet", gamma=gamma, precision=mixed[0])
    setup_s = time.perf_counter() - t0
    q = G.q
    log("setup (assembly + eigen-decompositions + upload): %.2f s, q = %d" % (setup_s, q))
    F = elliptic_batch(G.n, gamma, B, sigma=1e-3, seed0=1234)
    Fd = torch.from_numpy(F).cuda()
    rhs = torch.empty((B, q, q), dtype=torch.float64, device="cuda")
    U = torch.zeros((B, q, q), dtype=torch.float64, device="cuda")
    ws = mf.pcg_workspace(G.op, G.prec, B)

    def step(flags):
        G.rhs_op.apply(Fd, Y=rhs)
        return mf.pcg_solve(G.op, G.prec, rhs, U, tol=args.tol, maxit=300,
                            flags=flags | mf.PCG_ZERO_GUESS, workspace=ws)

    def timed(nsteps, flags, classes):
        # HIP events around the launches of the traced classes only (each
        # recorded launch costs the device a few microseconds between kernels)
        torch.cuda.synchronize()
        mf.trace_select(classes)
        mf.trace_enable(True)
        t = time.perf_counter()
        out = None
        for _ in range(nsteps):
            out = step(flags)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        mf.trace_enable(False)
        mf.trace_select(None)
        tr = {c: mf.trace_read(c) for c in range(mf.TRACE_CLASSES)}
        return dt, out, tr

    # ---- mixed path (headline) ---------------------------------------------------
    G.prec.set_precision(mixed[0])
    for _ in range(args.warmup):
        step(mf.PCG_FLEXIBLE)
    dt_mx, (it_mx, rr_mx, _), tr_mx = timed(args.steps, mf.PCG_FLEXIBLE, (mf.TRACE_BAND, mixed[1]))
    U_mixed0 = U[0].cpu().numpy()
    value = B * args.steps / dt_mx
    log("mixed: %.3f s/step, iterations %s, max relres %.2e" % (dt_mx / args.steps, it_mx.tolist(), rr_mx.max()))

    # ---- FP64 path -------------------------------------------------------------
    fp64 = None
    if args.fp64_steps > 0:
        G.prec.set_precision(mf.PREC_F64)
        step(0)
        dt_64, (it_64, rr_64, _), tr_64 = timed(args.fp64_steps, 0, (mf.TRACE_GEMM_F64,))
        fp64_value = B * args.fp64_steps / dt_64
        log("fp64: %.3f s/step, iterations %s, max relres %.2e"
            % (dt_64 / args.fp64_steps, it_64.tolist(), rr_64.max()))
        f_ms, f_n, f_items = tr_64[mf.TRACE_GEMM_F64]
        f64_tf = 2.0 * q ** 3 * f_items / (f_ms * 1e-3) / 1e12 if f_ms > 0 else 0.0
        fp64 = {"fp64_solves_per_s": round(fp64_value, 3),
                "mixed_over_fp64": round(value / fp64_value, 3),
                "iterations_fp64": int(it_64.max()),
                "relres_max_fp64": float(rr_64.max()),
                "gemm_f64": {"bound": "mfma", "achieved": round(f64_tf, 2), "peak": F64_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(f64_tf / F64_PEAK_TFLOPS, 4),
                             "avg_launch_ms": round(f_ms / max(f_n, 1), 4)}}

    # ---- FP64-accurate transforms from exact INT8 digit products --------------------
    int8 = None
    if args.int8_steps > 0:
        G.prec.set_precision(mf.PREC_F64_INT8)
        step(0)
        dt_i8, (it_i8, rr_i8, _), tr_i8 = timed(args.int8_steps, 0, (mf.TRACE_GEMM_I8,))
        i8_value = B * args.int8_steps / dt_i8
        log("fp64 via int8 digits: %.3f s/step, iterations %s, max relres %.2e"
            % (dt_i8 / args.int8_steps, it_i8.tolist(), rr_i8.max()))
        i_ms, i_n, i_items = tr_i8[mf.TRACE_GEMM_I8]
        # 28 digit products of 2 q^3 integer operations per item and launch
        i8_tops = 28 * 2.0 * q ** 3 * i_items / (i_ms * 1e-3) / 1e12 if i_ms > 0 else 0.0
        int8 = {"fp64_int8_solves_per_s": round(i8_value, 3),
                "iterations_fp64_int8": int(it_i8.max()),
                "relres_max_fp64_int8": float(rr_i8.max()),
                "gemm_i8": {"bound": "mfma", "achieved": round(i8_tops, 2), "peak": I8_PEAK_TOPS, "unit": "TOP/s",
                            "frac": round(i8_tops / I8_PEAK_TOPS, 4), "ops_count": "28 INT8 products of 2 q^3 per item",
                            "avg_launch_ms": round(i_ms / max(i_n, 1), 4)}}
        G.prec.set_precision(mixed[0])

    # ---- roofline of the dominant kernel in the timed region ---------------------
    # (the split back transform: the largest per-iteration kernel time of the
    # mixed path in the rocprofv3 summary; only it and the operator are traced)
    flop_per_item_gemm = 2.0 * q * q * q            # one transform product per item
    g_ms, g_n, g_items = tr_mx[mixed[1]]
    mfma_flop = mixed[2] * flop_per_item_gemm * g_items   # BF16 products per transform
    achieved_tf = mfma_flop / (g_ms * 1e-3) / 1e12 if g_ms > 0 else 0.0
    b_ms, b_n, b_items = tr_mx[mf.TRACE_BAND]
    op_bytes = 16.0 * q * q * b_items                # read X, write Y (FP64)
    op_gbs = op_bytes / (b_ms * 1e-3) / 1e9 if b_ms > 0 else 0.0
    log("trace mixed (ms): band %.1f gemm %.1f | avg gemm launch %.3f ms, avg band launch %.3f ms"
        % (b_ms, g_ms, g_ms / max(g_n, 1), b_ms / max(b_n, 1)))
    roofline = dict(bound="mfma", achieved=round(achieved_tf, 2), peak=BF16_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved_tf / BF16_PEAK_TFLOPS, 4),
                    traffic=measured_traffic(args.mixed, q, B),
                    traffic_unit="HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                    # the survey's per-unit count for this transform precision:
                    # mixed[2] BF16 MFMA products of 2 q^3 per item (the split
                    # issues three BF16 products for one FP32-accurate product)
                    flop_per_launch=mixed[2] * flop_per_item_gemm * g_items / max(g_n, 1),
                    flop_count="%d BF16 products of 2 q^3 per item" % mixed[2],
                    # the same launches counted as the method's one product per item
                    one_product_flop_per_launch=flop_per_item_gemm * g_items / max(g_n, 1),
                    one_product_frac=round(achieved_tf / mixed[2] / BF16_PEAK_TFLOPS, 4),
                    kernel=mixed[3] + " (transform product, %d BF16 MFMA products)" % mixed[2],
                    avg_launch_ms=round(g_ms / max(g_n, 1), 4), launches=g_n,
                    traced_classes="operator apply and this kernel only (HIP events on the launch stream)")

    extra = {}
    if args.heat_steps > 0:
        for i, hp in enumerate(args.heat_prec.split(",")):
            r = heat_leg(mf, torch, np, args.heat_steps, max(args.imex_steps, 2), hp)
            extra.update(r if i == 0 else {"imex_heat_p4_" + hp: r["imex_heat_p4"]})
    if args.dib_steps > 0:
        extra.update(dib_leg(mf, torch, np, args.dib_steps))
    if args.adjoint > 0:
        extra.update(adjoint_leg(mf, torch, np))
    if args.uneven > 0:
        extra.update(uneven_leg(mf, torch, np, args.uneven, mixed[0], args.mixed))
    if args.paper_prec > 0:
        extra.update(paper_prec_leg(mf, torch, np, G, B, max(args.imex_steps, 3)))

    # ---- CPU baseline (oracle) ----------------------------------------------------------
    cpu = None
    fwd = back = None
    if not args.no_cpu_baseline:
        cpu, fwd, back = cpu_baseline(F[0], k, m, gamma, args.tol, U_mixed0)
        log("oracle: %.4f solves/s (%s); GPU item 0 vs oracle: forward %.2e backward %.2e"
            % (cpu["value"], cpu["sample"], fwd, back))

    line = {
        "metric": "MO-PCG solves/s at N=2049 P2, rel 1e-8; mixed vs FP64 on same GPU; HBM GB/s",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt_mx / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 recurrence + %s (fp32 accumulate) transforms" % args.mixed,
        "data": "synthetic",
        "config": {"workload": "elliptic P2 x-normal, n=2049 (q=2047), Dirichlet, gamma=1, "
                               "manufactured f + 1e-3 noise, batch %d, rel residual %.0e" % (B, args.tol),
                   "global_batch": B, "parallelism": "batch on 1 GPU"},
        "iterations_mixed": int(it_mx.max()),
        "relres_max_mixed": float(rr_mx.max()),
        "setup_s": round(setup_s, 2),
        "op_apply": {"bound": "hbm", "achieved": round(op_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(op_gbs / HBM_PEAK_GBS, 4), "avg_launch_ms": round(b_ms / max(b_n, 1), 4)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "oracle_forward_err_item0": fwd,
        "oracle_backward_err_item0": back,
    }
    if fp64:
        line.update(fp64)
    if int8:
        line.update(int8)
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
