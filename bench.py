"""Benchmark of the DG-AMR hot path on one MI355X.

Workload (headline): the density current -- 25.6 x 1.6 x 6.4 km, 64 x 4 x 16
base hexes, N = 4, cold cosine bell -15 K with radii 4 km x 2 km at x = 0,
z = 3 km, refined two levels where |grad theta| > 1e-3 K/m with 2:1 balance,
no-flux walls; SSP-RK3 with dt = 0.01 s and an adaptation cycle every 10
steps (indicator, coarsen pass and projection, refine pass and projection)
inside the timed region.  The host part of a cycle (flag download, forest
passes) overlaps a step computed at once on the current mesh, kept when the
cycle changes no leaf and made again on the adapted mesh otherwise (the same
result either way).  One benchmark step = one SSP-RK3 step (3 fused stage
launches, each behind a mortar pre-pass).

Prints one JSON line: DOF-updates/s (5 variables x nodes x 3 RHS evaluations
per step) over the timed steps; the roofline of the dominant kernel pair (the
mortar pre-pass and the fused stage kernel of one dg_rk_stage call) from HIP
events around the stage launches of a second pass of as many steps (the timed
steps carry no events between stages: each timing marker costs the GPU a few
microseconds); the oracle timed on the host cores on one SSP-RK3 stage of the
same workload (1 thread and all cores, median of 3), with the other
configurations' oracle timings and the library-vs-oracle errors of that stage
(float64 and the precision split).  The AMR warm bubble (N = 7) and the other
workloads are in "extras".
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_STAGE_FIRST = 80.0       # per node: read qs (40 B), write qout (40 B); a = 0
BYTES_STAGE = 120.0            # per node: read q0 and qs, write qout
STAGE_KERNEL = {"density_current": "k_mortar<4, false> + k_stage<4, 2, false>",
                "amr_bubble": "k_mortar<7, false> + k_stage<7, 1, false>"}

# Density current: 25.6 x 1.6 x 6.4 km, 64 x 4 x 16 roots, N = 4, two levels on |grad theta|
DC = dict(N=4, nroot=(64, 4, 16), L=2, lo=(0.0, 0.0, 0.0), hi=(25600.0, 1600.0, 6400.0),
          bell=(-15.0, (0.0, 800.0, 3000.0), (4000.0, 0.0, 2000.0)), thr=1e-3, dt=0.01)
# AMR warm bubble: 1000 m box, 8^3 roots, N = 7, two levels on |theta'|
BUBBLE = dict(N=7, nroot=(8, 8, 8), L=2, lo=(0.0, 0.0, 0.0), hi=(1000.0, 1000.0, 1000.0),
              bell=(2.0, (500.0, 500.0, 350.0), (250.0, 250.0, 250.0)), thr=0.1, dt=0.001)

# Bytes beyond L2 per stage (the mortar pre-pass plus the fused stage kernel, the two
# launches of one dg_rk_stage call) over the stage-timing steps of the default run,
# from two counter runs of this command (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch, the two kernels summed), each scaled by the ratio of the bytes a plain
# device copy of known size moves to what the same counter reads for it.  Valid only
# for the kernel and forest sources they were taken on (SHA-256 below); otherwise
# traffic is reported as null.  Not measured by the run that prints the line.
TRAFFIC = {
    "sources_sha256": "a992e2f8746d593c2077687dadefb5f8294b1351ed84eb3e36473cabf9954e2a",
    "fetch_scale": 1048576.0 / 524299.5,  # 1 GiB copy: FETCH_SIZE reads 524299.5 KiB
    "write_scale": 1048576.0 / 1048576.0,  # 1 GiB copy: WRITE_SIZE reads 1048576.0 KiB
    "density_current": {"fetch_kib": 131085.2, "write_kib": 128877.3},
    "source": "profiles/k_stage_density_current_N4_traffic.md",
}
CSRC = os.path.join(ROOT, "paper_2404_16648_amd", "csrc")


def kernel_sources_sha256():
    """SHA-256 of the stage kernel's sources and of the forest (the leaf order sets
    the memory access pattern), or None if they cannot be delimited."""
    import hashlib
    with open(os.path.join(CSRC, "kernels.hip")) as f:
        src = f.read()
    a = src.find("// ---------------------------------------------------------------- adjoint")
    parts = [src[:a]] if a >= 0 else []
    for name in ("hipError_t launch_stage(", "hipError_t launch_mortar("):
        b = src.find(name)
        c = src.find("\n}\n", b)
        if b < 0 or c < 0:
            return None
        parts.append(src[b:c])
    if a < 0:
        return None
    h = hashlib.sha256()
    for part in parts:
        h.update(part.encode())
    for name in ("kernels.hpp", "device_common.hpp", "facetypes.hpp", "forest.cpp"):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_bytes_per_launch(workload="density_current"):
    t = TRAFFIC
    w = t[workload]
    if t["sources_sha256"] is None or t["sources_sha256"] != kernel_sources_sha256() or w["fetch_kib"] is None:
        return None
    return 1024.0 * (w["fetch_kib"] * t["fetch_scale"] + w["write_kib"] * t["write_scale"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--adapt-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--rtb-seconds", type=float, default=100.0,
                    help="simulated time of the rising-thermal-bubble long run in the extras (0: skip it; "
                         "counter passes skip it)")
    ap.add_argument("--acoustic-hours", type=float, default=18.0,
                    help="simulated hours of the two acoustic-wave runs on the shell in the extras (0: skip "
                         "them; counter passes skip them)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the timed steps, run 4 plain device copies of MIB MiB each "
                         "(reference launches for the memory-traffic counters)")
    return ap.parse_args()


def _progress(what):
    print(f"[bench] {what}", file=sys.stderr, flush=True)


def adaptive_run(dg, torch, cfg, steps, warmup, every):
    """SSP-RK3 with an adaptation cycle every `every` steps on the workload cfg:
    `steps` timed steps without events (throughput), then `steps` more with one
    event pair around the three stage launches of each step (stage duration)."""
    ph = dg.PhysParams()
    kind = dg.DG_IND_GRAD_THETA if cfg is DC else dg.DG_IND_THETA
    mesh, q = dg.initial_mesh(cfg["N"], cfg["nroot"], cfg["L"], cfg["lo"], cfg["hi"], (0, 0, 0), ph, cfg["bell"],
                              kind, cfg["thr"])
    stream = torch.cuda.current_stream()
    stepper = dg.AdaptiveStepper(mesh, ph, q, cfg["dt"], every, kind, cfg["thr"])
    state = {"dofs": 0}

    def one_step(record):
        ev = [] if record is not None else None
        stepper.step(ev)
        nodes = stepper.mesh.K * stepper.mesh.Np
        if record is not None:
            e0, e1 = ev[0]
            record.append((e0, e1, nodes * (BYTES_STAGE_FIRST + 2 * BYTES_STAGE), 3))
        state["dofs"] += 3 * 5 * nodes

    for _ in range(warmup):
        one_step(None)
    torch.cuda.synchronize()
    state["dofs"] = 0
    cycles0, changed0 = stepper.cycles, stepper.changed
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(steps):
        one_step(None)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    dofs = state["dofs"]
    cycles, changed = stepper.cycles - cycles0, stepper.changed - changed0
    events = []
    for _ in range(steps):
        one_step(events)
    torch.cuda.synchronize()
    stage_ms = sum(e0.elapsed_time(e1) for e0, e1, _, _ in events)
    stage_bytes = sum(b for _, _, b, _ in events)
    n_launches = sum(n for _, _, _, n in events)
    return {"stepper": stepper, "ph": ph, "dofs_per_s": dofs / (total_ms * 1e-3), "ms_per_step": total_ms / steps,
            "wall_s": wall, "stage_us": 1e3 * stage_ms / n_launches,
            "achieved_GBs": stage_bytes / (stage_ms * 1e-3) / 1e9, "alg_bytes_per_launch": stage_bytes / n_launches,
            "cycles": cycles, "changed": changed}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only (no multi-GPU path); use --gpus 1"}))
        sys.exit(2)
    import torch

    from paper_2404_16648_amd import dg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    _progress("density current: warm-up, timed steps, stage-timing steps")
    r = adaptive_run(dg, torch, DC, args.steps, args.warmup, args.adapt_every)
    stepper, ph = r["stepper"], r["ph"]
    m = stepper.mesh
    budgets = dg.dg_budgets(m, ph, stepper.q)
    calib = None
    if args.copy_calibration > 0:
        nb = args.copy_calibration << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        calib = {"bytes_per_copy": nb, "copies": 4}
        del src, dst
    traffic = traffic_bytes_per_launch("density_current")
    alg = r["alg_bytes_per_launch"]
    result = {
        "metric": "DG RHS DOF-updates/s (FP64)",
        "value": r["dofs_per_s"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "node_updates_per_s": r["dofs_per_s"] / 5.0,
        "dtype": "f64",
        "data": "synthetic (analytic density-current initial state)",
        "config": {"workload": "density current: 25.6 x 1.6 x 6.4 km, 64x4x16 base hexes, N=4, cold bell -15 K "
                               "(4 km x 2 km at x=0, z=3 km), 2 levels where |grad theta| > 1e-3 K/m, walls, "
                               "SSP-RK3 dt=0.01 s, adapt every 10 steps",
                   "leaves": m.K, "nodes": m.K * m.Np, "hanging_faces": int(m.info.n_hang),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": r["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r["achieved_GBs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "B/launch", "traffic_measured_in_this_run": False,
                     "traffic_source": TRAFFIC["source"] + " (rocprofv3 --pmc FETCH_SIZE, WRITE_SIZE of this command)",
                     "algorithmic_bytes_per_launch": alg,
                     "traffic_over_algorithmic": None if traffic is None else traffic / alg,
                     "kernel": STAGE_KERNEL["density_current"] +
                               " (mortar pre-pass, then fused volume+faces+lift+RK stage; one dg_rk_stage call)",
                     "avg_launch_us": r["stage_us"]},
        "wall_s": r["wall_s"],
        "mass_prime_final": budgets[0],
        "adaptation_cycles": {"run": r["cycles"], "changed_mesh": r["changed"]},
    }
    if calib is not None:
        result["copy_calibration"] = calib
    if not args.no_extras:
        result["extras"] = extras(dg, torch, stepper.mesh, stepper.q, ph, args)
    if not args.no_cpu_baseline:
        _progress("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(dg, torch)
    print(json.dumps(result), flush=True)


def _time_launches(torch, fn, reps, warmup=5, batches=5):
    """Duration (us) of one fn(): HIP events on the current stream around batches
    of reps back-to-back calls (no timing marker between two calls), the median
    batch divided by reps."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    d = []
    for _ in range(batches):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        d.append(1e3 * e0.elapsed_time(e1) / reps)
    d.sort()
    return d[len(d) // 2]


def _cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def forced_cycle(dg, torch, mesh, q, reps=5):
    """AMR transfer on a forced cycle: coarsen every family of finest leaves, project,
    refine those parents back, project.  Host pass time and projection kernels."""
    import numpy as np
    lev = mesh.tables()["leaf"][:, 1]
    flc = np.where(lev == lev.max(), -1, 0).astype(np.int8)
    host_c, host_r, kc, kr = [], [], [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mc = dg.dg_mesh_build(prev=mesh, flags=flc, pass_=dg.DG_PASS_COARSEN)
        t1 = time.perf_counter()
        qc = mc.field()
        kc.append(_time_launches(torch, lambda: dg.dg_coarsen_project(mesh, mc, q, qc), 20))
        flr = np.where(mc.tables()["xfer_kind"] == dg.DG_KIND_FAMILY, 1, 0).astype(np.int8)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        mr = dg.dg_mesh_build(prev=mc, flags=flr, pass_=dg.DG_PASS_REFINE)
        t3 = time.perf_counter()
        qr = mr.field()
        kr.append(_time_launches(torch, lambda: dg.dg_refine_project(mc, mr, qc, qr), 20))
        host_c.append(1e3 * (t1 - t0))
        host_r.append(1e3 * (t3 - t2))
    med = lambda v: sorted(v)[len(v) // 2]
    np_ = mesh.Np
    bytes_c = 40.0 * np_ * (mesh.K + mc.K)   # read every source leaf, write every target leaf
    bytes_r = 40.0 * np_ * (mc.K + mr.K)
    return {"leaves": [mesh.K, mc.K, mr.K], "families": int(mc.info.n_coarsened),
            "coarsen_pass_host_ms": med(host_c), "refine_pass_host_ms": med(host_r),
            "coarsen_project_us": med(kc), "refine_project_us": med(kr),
            "coarsen_project_GBs": bytes_c / (med(kc) * 1e-6) / 1e9,
            "refine_project_GBs": bytes_r / (med(kr) * 1e-6) / 1e9,
            "coarsen_frac_hbm": bytes_c / (med(kc) * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "refine_frac_hbm": bytes_r / (med(kr) * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "same_leaves_after_cycle": bool(mr.K == mesh.K)}


def rtb_long_run(dg, torch, t_end=100.0, regrid=25.0, dt=0.0025, seg=100, mu=1.5):
    """Rising-thermal-bubble-style long run (section 4.3's setting, quasi-2-D: 1000 m x
    1000 m in x, z, one 100 m root periodic along y; 10 x 1 x 10 roots, N = 4, two
    levels where |theta'| > 0.05 K, warm bubble 0.5 K, radius 250 m at (500, 350) m,
    walls in x and z; artificial viscosity mu = 1.5 m^2/s as in that section), SSP-RK3 with a regrid every `regrid`
    seconds.  Steps between regrids run as replays of a HIP graph of `seg` steps; a
    progress line goes to stderr at every regrid.  Reports the relative change of
    the total mass and energy over the run."""
    if t_end <= 0:
        return {"skipped": True}
    ph = dg.PhysParams(mu=mu)
    thr = 0.05
    mesh, q = dg.initial_mesh(4, (10, 1, 10), 2, (0.0, 0.0, 0.0), (1000.0, 100.0, 1000.0), (0, 1, 0), ph,
                              (0.5, (500.0, 50.0, 350.0), (250.0, 0.0, 250.0)), dg.DG_IND_THETA, thr)
    b0 = dg.dg_budgets(mesh, ph, q)
    steps_per_regrid = int(round(regrid / dt))
    nreg = int(round(t_end / regrid))
    leaves, t0 = [mesh.K], time.perf_counter()
    steps = 0
    for c in range(nreg):
        if c > 0:
            m2, q = dg.adapt_cycle(mesh, ph, q, dg.DG_IND_THETA, thr)
            m2.prev = None
            mesh = m2
            leaves.append(mesh.K)
        g = dg.GraphedSteps(mesh, ph, dt, q, seg)
        for _ in range(steps_per_regrid // seg):
            g.replay()
        q = g.q
        steps += steps_per_regrid // seg * seg
        del g
        try:
            b1 = dg.dg_budgets(mesh, ph, q)
        except dg.DGError as err:  # a non-finite state ends the run
            return {"t_end_s": t_end, "dt_s": dt, "steps": steps, "non_finite_by_s": steps * dt, "error": str(err)}
        _progress(f"long run: t = {steps * dt:.0f} s of {t_end:.0f} s, {mesh.K} leaves, "
                  f"mass change {(b1[1] - b0[1]) / b0[1]:.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"t_end_s": t_end, "regrid_s": regrid, "dt_s": dt, "mu_m2_s": mu, "steps": steps, "regrids": nreg - 1,
            "leaves_min_max": [min(leaves), max(leaves)], "wall_s": wall,
            "mass_rel_change": (b1[1] - b0[1]) / b0[1], "energy_rel_change": (b1[3] - b0[3]) / abs(b0[3])}


# bytes per node of one shell stage with a != 0: q0, the stage input and the output
# (120), the Jacobian and nine metric terms (80), the face normals and face Jacobians
# of the element's 6 (N+1)^2 face nodes (6 x 25 x 32 / 125 = 38.4 at N = 4)
def sphere_bytes_per_node(N):
    n1 = N + 1
    return 120.0 + 80.0 + 6.0 * n1 * n1 * 32.0 / n1 ** 3


def sphere_shell(dg, torch, N=4, n=24, nz=8, dt=0.1, steps=10):
    """Cubed-sphere shell of section 4.4's size (6 panels of 24 x 24 elements, 8
    layers, N = 4, r_e = 6371 km, 10 km top; uniform, no refinement), isothermal
    300 K background, a Gaussian theta' of 1 K and 500 km half-width at latitude 0,
    longitude 0: stage and right-hand-side durations, the HBM fraction of the stage
    and the mass change over SSP-RK3 steps."""
    ph = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL)
    m = dg.dg_sphere_mesh_build(N, n, nz)
    xyz = torch.empty(3, m.K, m.Np, dtype=torch.float64, device="cuda")
    dg.dg_node_coords(m, xyz)
    r = torch.sqrt(xyz[0] ** 2 + xyz[1] ** 2 + xyz[2] ** 2)
    r_e, R, T0 = 6.371e6, ph.cp - ph.cv, ph.theta0
    rho_b = ph.P0 * torch.exp(-ph.g * (r - r_e) / (R * T0)) / (R * T0)
    dist = r_e * torch.arccos(torch.clamp(xyz[0] / r, -1.0, 1.0))
    q = m.field()
    q[4] = rho_b * torch.exp(-(dist / 5.0e5) ** 2)
    del xyz, r, rho_b, dist
    qs, q1 = torch.empty_like(q), torch.empty_like(q)
    dg.dg_rk_stage(m, ph, 0.0, 1.0, dt, q, q, qs)
    nodes = m.K * m.Np
    st_us = _time_launches(torch, lambda: dg.dg_rk_stage(m, ph, 0.75, 0.25, dt, q, qs, q1), 20)
    R1 = torch.empty_like(q)
    rhs_us = _time_launches(torch, lambda: dg.dg_rhs(m, ph, q, R1), 20)
    bpn = sphere_bytes_per_node(N)
    b0 = dg.dg_budgets(m, ph, q)
    a, b = torch.empty_like(q), torch.empty_like(q)
    x = q.clone()
    for _ in range(steps):
        dg.ssp_rk3_step(m, ph, dt, x, a, b)
    b1 = dg.dg_budgets(m, ph, x)
    return {"workload": "cubed-sphere shell 6 x 24 x 24 x 8, N=4, r_e 6371 km, top 10 km, isothermal 300 K, "
                        "theta' Gaussian 1 K / 500 km, SSP-RK3 dt=0.1 s",
            "leaves": m.K, "nodes": nodes, "kernel": "k_stage_sphere<4, 1>",
            "stage_us": st_us, "rhs_us": rhs_us, "bytes_per_node": bpn,
            "frac_hbm": nodes * bpn / (st_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "dof_updates_per_s": 5.0 * nodes / (st_us * 1e-6),
            "mass_prime_change_10_steps_rel_mass": (b1[0] - b0[0]) / b0[1],
            "energy_rel_change_10_steps": (b1[3] - b0[3]) / abs(b0[3])}


def shell_transfers(dg, torch, N=4, n=12, nz=4):
    """Section 3.4's transfer between the shell 6 x n x n x nz and its refinement
    6 x 2n x 2n x 2nz (the shell of sphere_shell): refinement (reference
    interpolation, the two mass reductions and the scale factor) and coarsening
    (reference projections and the volume-weighted mean) durations, the scale
    factor, the volume loss (isoparametric volumes) and the mass change of each
    transfer, on the Gaussian theta' state of sphere_shell."""
    ph = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL)
    mc, mf = dg.dg_sphere_mesh_build(N, n, nz), dg.dg_sphere_mesh_build(N, 2 * n, 2 * nz)
    xyz = torch.empty(3, mc.K, mc.Np, dtype=torch.float64, device="cuda")
    dg.dg_node_coords(mc, xyz)
    r = torch.sqrt(xyz[0] ** 2 + xyz[1] ** 2 + xyz[2] ** 2)
    r_e, R, T0 = 6.371e6, ph.cp - ph.cv, ph.theta0
    rho_b = ph.P0 * torch.exp(-ph.g * (r - r_e) / (R * T0)) / (R * T0)
    dist = r_e * torch.arccos(torch.clamp(xyz[0] / r, -1.0, 1.0))
    qc = mc.field()
    qc[4] = rho_b * torch.exp(-(dist / 5.0e5) ** 2)
    del xyz, r, rho_b, dist
    qf, qc2 = mf.field(), mc.field()
    s = dg.dg_sphere_refine_project(mc, mf, ph, qc, qf)
    b0, b1 = dg.dg_budgets(mc, ph, qc), dg.dg_budgets(mf, ph, qf)
    dg.dg_sphere_coarsen_project(mf, mc, ph, qf, qc2)
    b2 = dg.dg_budgets(mc, ph, qc2)
    ref_us = _time_launches(torch, lambda: dg.dg_sphere_refine_project(mc, mf, ph, qc, qf, scale=False), 10)
    crs_us = _time_launches(torch, lambda: dg.dg_sphere_coarsen_project(mf, mc, ph, qf, qc2), 10)
    _, (vc, _) = dg.dg_sphere_volumes(mc)
    _, (vf, ve) = dg.dg_sphere_volumes(mf)
    byt = 40.0 * (mc.K + mf.K) * mc.Np      # one read of the source, one write of the target
    return {"workload": f"6 x {n} x {n} x {nz} <-> 6 x {2 * n} x {2 * n} x {2 * nz}, N={N}, isothermal, "
                        "theta' Gaussian 1 K / 500 km",
            "refine_us": ref_us, "coarsen_us": crs_us,
            "refine_note": "k_shell_refine + two mass reductions + k_shell_scale",
            "coarsen_GBs": byt / (crs_us * 1e-6) / 1e9,
            "scale_factor_minus_1": s - 1.0,
            "volume_loss_rel": vf / vc - 1.0, "fine_volume_vs_spherical_excess_rel": vf / ve - 1.0,
            "refine_mass_change_rel": (b1[1] - b0[1]) / b0[1],
            "coarsen_mass_change_rel": (b2[1] - b1[1]) / b1[1]}


def acoustic_wave(dg, torch, N=4, n=12, nz=1, dt=0.9, hours=18.0):
    """Section 4.4's acoustic wave as the paper's two-dimensional shallow-atmosphere
    problem (no gravity, uniform 300 K background): a cosine bell of 100 Pa and
    radius r_e/3 about latitude 0, longitude 0 times sin(pi h / H), potential
    temperature unperturbed; SSP-RK3 on 6 x n x n x nz.  Reports when the pressure
    pulse at the antipode (mean over the nodes within 300 km) crosses zero between
    its positive and negative lobes, against pi r_e / c, and the mass and energy
    change over the run."""
    import math
    ph = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL, g=0.0)
    m = dg.dg_sphere_mesh_build(N, n, nz)
    xyz = torch.empty(3, m.K, m.Np, dtype=torch.float64, device="cuda")
    dg.dg_node_coords(m, xyz)
    r = torch.sqrt(xyz[0] ** 2 + xyz[1] ** 2 + xyz[2] ** 2)
    r_e, H, R, T0, P0 = 6.371e6, 1.0e4, ph.cp - ph.cv, ph.theta0, ph.P0
    gam = ph.cp / ph.cv
    dist = r_e * torch.arccos(torch.clamp(xyz[0] / r, -1.0, 1.0))
    r_c = r_e / 3.0
    f = torch.where(dist <= r_c, 50.0 * (1.0 + torch.cos(math.pi * dist / r_c)), torch.zeros_like(dist))
    pp = f * torch.sin(math.pi * (r - r_e) / H)
    Thb = P0 / R                                   # uniform background: P = P0, rho = P0 / (R T0)
    q = m.field()
    q[4] = (P0 / R) * ((P0 + pp) / P0) ** (1.0 / gam) - Thb
    q[0] = q[4] / T0
    anti = r_e * torch.arccos(torch.clamp(-xyz[0] / r, -1.0, 1.0)) <= 3.0e5
    idx = torch.nonzero(anti.reshape(-1)).reshape(-1)
    del xyz, r, dist, f, pp, anti
    a, b = m.field(), m.field()
    b0 = dg.dg_budgets(m, ph, q)
    every, t_first = 300.0, 14.0 * 3600.0
    times, vals = [], []
    t, steps, nxt = 0.0, 0, t_first
    t0 = time.perf_counter()
    while t < hours * 3600.0 - 1e-9:
        dg.ssp_rk3_step(m, ph, dt, q, a, b)
        t += dt
        steps += 1
        if t >= nxt - 1e-9:
            thp = q[4].reshape(-1)[idx]
            times.append(t)
            vals.append(float((P0 * ((R * (Thb + thp) / P0) ** gam - 1.0)).mean()))
            nxt += every
        if steps % 20000 == 0:
            _progress(f"acoustic wave: t = {t / 3600.0:.1f} h")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b1 = dg.dg_budgets(m, ph, q)
    i_max = max(range(len(vals)), key=lambda i: vals[i])
    j = next((k for k in range(i_max, len(vals)) if vals[k] < 0.0), None)
    t_zero = None if j is None else times[j - 1] + every * vals[j - 1] / (vals[j - 1] - vals[j])
    c = math.sqrt(gam * R * T0)
    return {"workload": f"cubed-sphere shell 6 x {n} x {n} x {nz}, N={N}, no gravity, 300 K, bell 100 Pa, "
                        f"r_c = r_e/3, SSP-RK3 dt={dt} s, {hours} h",
            "steps": steps, "wall_s": wall, "antipode_max_Pa": max(vals), "antipode_min_Pa": min(vals),
            "antipode_zero_crossing_h": None if t_zero is None else t_zero / 3600.0,
            "pi_r_e_over_c_h": math.pi * r_e / c / 3600.0, "c_m_s": c,
            "mass_rel_change": (b1[1] - b0[1]) / b0[1], "energy_rel_change": (b1[3] - b0[3]) / abs(b0[3])}


def _acoustic_state(dg, torch, m, ph, xyz):
    """section 4.4's acoustic initial state without gravity (uniform 300 K
    background): P' = bell(100 Pa, r_e/3) x sin(pi h / H), theta unperturbed"""
    import math
    r = torch.sqrt(xyz[0] ** 2 + xyz[1] ** 2 + xyz[2] ** 2)
    r_e, H, R, T0, P0 = 6.371e6, 1.0e4, ph.cp - ph.cv, ph.theta0, ph.P0
    gam = ph.cp / ph.cv
    dist = r_e * torch.arccos(torch.clamp(xyz[0] / r, -1.0, 1.0))
    r_c = r_e / 3.0
    f = torch.where(dist <= r_c, 50.0 * (1.0 + torch.cos(math.pi * dist / r_c)), torch.zeros_like(dist))
    pp = f * torch.sin(math.pi * (r - r_e) / H)
    q = m.field()
    q[4] = (P0 / R) * ((P0 + pp) / P0) ** (1.0 / gam) - P0 / R
    q[0] = q[4] / T0
    return q


def acoustic_wave_adaptive(dg, torch, N=4, n=12, nz=1, dt=0.45, hours=18.0, thr=5.0, regrid_h=1.0, seg=100):
    """Section 4.4's acoustic wave with adaptation: the 6 x n x n x nz shell may
    refine once (max_level 1; the oct-tree splits the layer too), regridded every
    hour on |P'| > thr (the pressure-perturbation criterion), steps between regrids
    replayed as HIP graphs of `seg` steps; no gravity (the paper's two-dimensional
    shallow-atmosphere problem).  Reports the antipode pulse's zero crossing against
    pi r_e / c, the leaf counts, and the total mass and energy change over the run,
    regrids included (the shell transfers keep the J W quadrature of the mass)."""
    import math
    ph = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL, g=0.0)
    m = dg.dg_sphere_mesh_build(N, n, nz, max_level=1)
    xyz = torch.empty(3, m.K, m.Np, dtype=torch.float64, device="cuda")
    dg.dg_node_coords(m, xyz)
    q = _acoustic_state(dg, torch, m, ph, xyz)
    fl = dg.dg_indicator(m, ph, q, dg.DG_IND_PPRIME, thr)
    fl[fl < 0] = 0
    m = dg.dg_mesh_build(prev=m, flags=fl, pass_=dg.DG_PASS_REFINE)
    m.prev = None
    xyz = torch.empty(3, m.K, m.Np, dtype=torch.float64, device="cuda")
    dg.dg_node_coords(m, xyz)
    q = _acoustic_state(dg, torch, m, ph, xyz)
    b0 = dg.dg_budgets(m, ph, q)
    R, P0, gam = ph.cp - ph.cv, ph.P0, ph.cp / ph.cv
    per_regrid = int(round(regrid_h * 3600.0 / dt)) // seg
    sample_every = max(1, int(round(270.0 / (seg * dt))))
    times, vals, leaves = [], [], [m.K]
    t, steps = 0.0, 0
    t0 = time.perf_counter()
    nreg = int(round(hours / regrid_h))
    for c in range(nreg):
        if c > 0:
            m2, q = dg.adapt_cycle(m, ph, q, dg.DG_IND_PPRIME, thr)
            m2.prev = None
            m = m2
            leaves.append(m.K)
        xyz = torch.empty(3, m.K, m.Np, dtype=torch.float64, device="cuda")
        dg.dg_node_coords(m, xyz)
        r = torch.sqrt(xyz[0] ** 2 + xyz[1] ** 2 + xyz[2] ** 2)
        anti = 6.371e6 * torch.arccos(torch.clamp(-xyz[0] / r, -1.0, 1.0)) <= 3.0e5
        idx = torch.nonzero(anti.reshape(-1)).reshape(-1)
        del xyz, r, anti
        g = dg.GraphedSteps(m, ph, dt, q, seg)
        for k in range(per_regrid):
            g.replay()
            t += seg * dt
            steps += seg
            if t >= 14.0 * 3600.0 and (k + 1) % sample_every == 0:
                thp = g.q[4].reshape(-1)[idx]
                times.append(t)
                vals.append(float((P0 * ((R * (P0 / R + thp) / P0) ** gam - 1.0)).mean()))
        q = g.q
        del g
        _progress(f"adaptive acoustic wave: t = {t / 3600.0:.0f} h, {m.K} leaves")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b1 = dg.dg_budgets(m, ph, q)
    i_max = max(range(len(vals)), key=lambda i: vals[i]) if vals else 0
    j = next((k for k in range(i_max, len(vals)) if vals[k] < 0.0), None)
    t_zero = None if j is None or j == 0 else times[j - 1] + (times[j] - times[j - 1]) * vals[j - 1] / (
        vals[j - 1] - vals[j])
    c = math.sqrt(gam * R * ph.theta0)
    return {"workload": f"cubed-sphere shell 6 x {n} x {n} x {nz}, N={N}, max_level 1, regrid every {regrid_h} h on "
                        f"|P'| > {thr} Pa, no gravity, 300 K, bell 100 Pa, SSP-RK3 dt={dt} s, {hours} h",
            "steps": steps, "regrids": nreg - 1, "leaves_min_max": [min(leaves), max(leaves)], "wall_s": wall,
            "antipode_max_Pa": max(vals) if vals else None,
            "antipode_zero_crossing_h": None if t_zero is None else t_zero / 3600.0,
            "pi_r_e_over_c_h": math.pi * 6.371e6 / c / 3600.0,
            "mass_rel_change": (b1[1] - b0[1]) / b0[1], "energy_rel_change": (b1[3] - b0[3]) / abs(b0[3])}


def sphere_shell_refined(dg, torch, N=4, n=24, nz=8, dt=0.05, thr=20.0):
    """The shell of sphere_shell refined once where the acoustic state's |P'| exceeds
    thr (section 4.4's regrid criterion; no gravity): stage duration with the mortar
    pre-pass of the hanging faces, and its HBM fraction at the shell's bytes per node."""
    ph = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL, g=0.0)
    m = dg.dg_sphere_mesh_build(N, n, nz, max_level=1)
    xyz = torch.empty(3, m.K, m.Np, dtype=torch.float64, device="cuda")
    dg.dg_node_coords(m, xyz)
    q = _acoustic_state(dg, torch, m, ph, xyz)
    fl = dg.dg_indicator(m, ph, q, dg.DG_IND_PPRIME, thr)
    fl[fl < 0] = 0
    mr = dg.dg_mesh_build(prev=m, flags=fl, pass_=dg.DG_PASS_REFINE)
    qr = mr.field()
    dg.dg_sphere_adapt_project(m, mr, ph, q, qr)
    del xyz, q
    qs, q1 = torch.empty_like(qr), torch.empty_like(qr)
    dg.dg_rk_stage(mr, ph, 0.0, 1.0, dt, qr, qr, qs)
    st_us = _time_launches(torch, lambda: dg.dg_rk_stage(mr, ph, 0.75, 0.25, dt, qr, qs, q1), 20)
    nodes = mr.K * mr.Np
    bpn = sphere_bytes_per_node(N)
    return {"workload": f"cubed-sphere shell 6 x {n} x {n} x {nz}, N={N}, refined once where |P'| > {thr} Pa of the "
                        "acoustic state, no gravity",
            "leaves": mr.K, "hanging_faces": mr.info.n_hang, "nodes": nodes,
            "kernels": "k_mortar_sphere<4> + k_stage_sphere<4, 1>", "stage_us": st_us, "bytes_per_node": bpn,
            "frac_hbm": nodes * bpn / (st_us * 1e-6) / 1e9 / HBM_PEAK_GBS}


def sphere_vortex(dg, torch, N=4, n=24, nz=8, thr=0.1, dt=0.1, steps=20):
    """The shell configuration of section 4.4's size with the isothermal 300 K
    atmosphere under gravity and a Gaussian theta vortex (1 K, 500 km, at latitude 0,
    longitude 0, at unperturbed density), refined once where theta' > thr: the
    float64 and precision-split stage durations and the split's error against the
    float64 stage (the library's float64 stage is held to the oracle at this size
    by the parity tests), the transposed right-hand side
    against the right-hand side, and the gradient of a final-time functional over
    `steps` checkpointed SSP-RK3 steps against the forward integration."""
    from paper_2404_16648_amd import adjoint as adj
    ph = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL)
    pm = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL, precision=dg.DG_MIXED)
    m = dg.dg_sphere_mesh_build(N, n, nz, max_level=1)

    def vortex(mesh):
        xyz = torch.empty(3, mesh.K, mesh.Np, dtype=torch.float64, device="cuda")
        dg.dg_node_coords(mesh, xyz)
        r = torch.sqrt(xyz[0] ** 2 + xyz[1] ** 2 + xyz[2] ** 2)
        r_e, R, T0 = 6.371e6, ph.cp - ph.cv, ph.theta0
        rho_b = ph.P0 * torch.exp(-ph.g * (r - r_e) / (R * T0)) / (R * T0)
        dist = r_e * torch.arccos(torch.clamp(xyz[0] / r, -1.0, 1.0))
        q = mesh.field()
        q[4] = rho_b * torch.exp(-(dist / 5.0e5) ** 2)
        return q

    fl = dg.dg_indicator(m, ph, vortex(m), dg.DG_IND_THETA, thr)
    fl[fl < 0] = 0
    mr = dg.dg_mesh_build(prev=m, flags=fl, pass_=dg.DG_PASS_REFINE)
    q = vortex(mr)
    del m
    q1, o64, o32 = torch.empty_like(q), torch.empty_like(q), torch.empty_like(q)
    dg.dg_rk_stage(mr, ph, 0.0, 1.0, dt, q, q, q1)
    st64 = _time_launches(torch, lambda: dg.dg_rk_stage(mr, ph, 0.75, 0.25, dt, q, q1, o64), 20)
    st32 = _time_launches(torch, lambda: dg.dg_rk_stage(mr, pm, 0.75, 0.25, dt, q, q1, o32), 20)
    # the split's error on the stage increment (the stage output minus its input)
    err = _field_err(torch, o32 - q1, o64 - q1)
    lam = torch.randn(q.shape, dtype=torch.float64, device=q.device, generator=torch.Generator(q.device).manual_seed(5))
    R, g = torch.empty_like(q), torch.empty_like(q)
    rhs_us = _time_launches(torch, lambda: dg.dg_rhs(mr, ph, q1, R), 20)
    adj_us = _time_launches(torch, lambda: dg.dg_rhs_adjoint(mr, ph, q1, lam, g), 20)
    gm = torch.empty_like(q)
    adjm_us = _time_launches(torch, lambda: dg.dg_rhs_adjoint(mr, pm, q1, lam, gm), 20)
    adj_err = _field_err(torch, gm, g)

    def gradient(phys):
        for rep in range(2):  # the first pass loads the kernels; the second is timed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x = q.clone().requires_grad_(True)
            qT = adj.integrate(x, mr, phys, dt, steps, 10)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            (gx,) = torch.autograd.grad(qT, x, grad_outputs=lam)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        return gx, t1 - t0, t2 - t1

    gx, fw, bw = gradient(ph)
    gxm, fwm, bwm = gradient(pm)
    finite = bool(torch.isfinite(gx).all())
    return {"workload": f"cubed-sphere shell 6 x {n} x {n} x {nz}, N={N}, isothermal 300 K under gravity, theta' "
                        f"Gaussian 1 K / 500 km, refined once where theta' > {thr} K",
            "leaves": mr.K, "hanging_faces": mr.info.n_hang, "nodes": mr.K * mr.Np,
            "stage_fp64_us": st64, "stage_mixed_us": st32, "mixed_speedup": st64 / st32,
            "mixed_stage_increment_rel_l2_vs_fp64(rho',momentum,Theta')": err,
            "rhs_us": rhs_us, "rhs_adjoint_us": adj_us, "adjoint_over_rhs": adj_us / rhs_us,
            "rhs_adjoint_mixed_us": adjm_us, "mixed_adjoint_speedup": adj_us / adjm_us,
            "mixed_adjoint_rel_l2_vs_fp64(rho',momentum,Theta')": adj_err,
            "gradient": {"steps": steps, "dt": dt, "checkpoint_every": 10, "forward_s": fw, "backward_s": bw,
                         "ratio": bw / fw, "finite": finite,
                         "mixed": {"forward_s": fwm, "backward_s": bwm, "ratio": bwm / fwm,
                                   "rel_l2_vs_fp64(rho',momentum,Theta')": _field_err(torch, gxm, gx)}}}


def budget_drift(dg, torch, mesh, q, ph, dt, steps=10):
    """Change of the integral of rho' per SSP-RK3 step over `steps` steps (no
    adaptation), relative to the integral of rho = rho_bar + rho'."""
    a, b = torch.empty_like(q), torch.empty_like(q)
    x = q.clone()
    b0 = dg.dg_budgets(mesh, ph, x)
    for _ in range(steps):
        dg.ssp_rk3_step(mesh, ph, dt, x, a, b)
    b1 = dg.dg_budgets(mesh, ph, x)
    return abs(b1[0] - b0[0]) / steps / abs(b0[1])


def _field_err(torch, a, b):
    out = []
    for sl in (slice(0, 1), slice(1, 4), slice(4, 5)):
        nb = float(torch.linalg.vector_norm(b[sl]))
        out.append(float(torch.linalg.vector_norm(a[sl] - b[sl])) / nb if nb > 0 else 0.0)
    return out


def extras(dg, torch, mesh, q, ph, args):
    """Precision split and adjoint costs on the headline mesh, the forced
    adaptation cycle there, the AMR warm bubble, the adjoint configuration, the
    uniform 4^3 case, the long run and the measured copy and FMA rates."""
    out = {}
    dt = DC["dt"]
    mixed = dg.PhysParams(precision=dg.DG_MIXED)
    _progress("extras: density current precision split and adjoint")
    qs = torch.empty_like(q)
    dg.dg_rk_stage(mesh, ph, 0.0, 1.0, dt, q, q, qs)      # a distinct stage input: q0 and qs both read
    q1 = torch.empty_like(q)
    nodes = mesh.K * mesh.Np
    f64_us = _time_launches(torch, lambda: dg.dg_rk_stage(mesh, ph, 0.75, 0.25, dt, q, qs, q1), 20)
    mixed_us = _time_launches(torch, lambda: dg.dg_rk_stage(mesh, mixed, 0.75, 0.25, dt, q, qs, q1), 20)
    Ra, Rb = torch.empty_like(q), torch.empty_like(q)
    dg.dg_rhs(mesh, ph, q, Ra)
    dg.dg_rhs(mesh, mixed, q, Rb)
    out["density_current_stage"] = {
        "stage_us_fp64": f64_us, "stage_us_mixed": mixed_us, "speedup_mixed": f64_us / mixed_us,
        "frac_hbm_fp64": nodes * BYTES_STAGE / (f64_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
        "frac_hbm_mixed": nodes * BYTES_STAGE / (mixed_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
        "mixed_rhs_rel_l2_vs_fp64_library(rho',momentum,Theta')": _field_err(torch, Rb, Ra),
        "mass_drift_per_step_rel_fp64": budget_drift(dg, torch, mesh, q, ph, dt),
        "mass_drift_per_step_rel_mixed": budget_drift(dg, torch, mesh, q, mixed, dt)}
    lam = torch.randn(q.shape, dtype=torch.float64, device=q.device, generator=torch.Generator(q.device).manual_seed(7))
    g = torch.empty_like(q)
    rhs_us = _time_launches(torch, lambda: dg.dg_rhs(mesh, ph, q, Ra), 20)
    adj_us = _time_launches(torch, lambda: dg.dg_rhs_adjoint(mesh, ph, q, lam, g), 20)
    out["density_current_adjoint_rhs"] = {"rhs_us": rhs_us, "rhs_adjoint_us": adj_us, "ratio": adj_us / rhs_us}
    # passive tracer (section 2.1's C = rho c) on the same mesh: its stage beside the Euler stage
    c0 = 1.0 + 0.1 * torch.rand(mesh.K, mesh.Np, dtype=torch.float64, device=q.device,
                                generator=torch.Generator(q.device).manual_seed(5))
    cs, c1 = c0.clone(), torch.empty_like(c0)
    tr_us = _time_launches(torch, lambda: dg.dg_tracer_stage(mesh, ph, 0.75, 0.25, dt, qs, c0, cs, c1), 20)
    out["density_current_tracer_stage"] = {
        "stage_us": tr_us, "bytes_per_node": 64.0, "kernels": "k_tracer_mortar<4, false> + k_tracer_stage<4, 1>",
        "note": "reads the Euler stage input (40 B/node) and c0, cs, writes the tracer (8 B each)",
        "frac_hbm": nodes * 64.0 / (tr_us * 1e-6) / 1e9 / HBM_PEAK_GBS}
    # a whole SSP-RK3 step of the Euler state and the tracer: the tracer stages on the
    # same stream as the Euler stages, or on a side stream beside them
    qq, cc = q.clone(), c0.clone()
    qa, qb, ca, cb = torch.empty_like(q), torch.empty_like(q), torch.empty_like(c0), torch.empty_like(c0)
    euler_us = _time_launches(torch, lambda: dg.ssp_rk3_step(mesh, ph, dt, qq, qa, qb), 10)
    one_us = _time_launches(torch, lambda: dg.ssp_rk3_step_tracer(mesh, ph, dt, qq, qa, qb, cc, ca, cb), 10)
    side = torch.cuda.Stream()
    two_us = _time_launches(torch, lambda: dg.ssp_rk3_step_tracer(mesh, ph, dt, qq, qa, qb, cc, ca, cb, side=side), 10)
    out["density_current_tracer_step"] = {
        "euler_step_us": euler_us, "euler_and_tracer_one_stream_us": one_us,
        "euler_and_tracer_side_stream_us": two_us, "side_stream_speedup": one_us / two_us,
        "tracer_cost_over_euler_step": (two_us - euler_us) / euler_us}
    del lam, g, Ra, Rb, q1, c0, cs, c1, qq, cc, qa, qb, ca, cb
    _progress("extras: density current forced adaptation cycle")
    out["density_current_forced_cycle"] = forced_cycle(dg, torch, mesh, q)
    # ---- AMR warm bubble (N = 7): the adaptive run as for the headline
    _progress("extras: AMR warm bubble")
    rb = adaptive_run(dg, torch, BUBBLE, 30, 5, 10)
    mb, qb = rb["stepper"].mesh, rb["stepper"].q
    out["amr_bubble"] = {"workload": "1000 m box, 8x8x8 base, N=7, 2 levels where |theta'| > 0.1 K, SSP-RK3 "
                                     "dt=0.001 s, adapt every 10 steps", "leaves": mb.K, "nodes": mb.K * mb.Np,
                         "hanging_faces": int(mb.info.n_hang), "dof_updates_per_s": rb["dofs_per_s"],
                         "ms_per_step": rb["ms_per_step"], "stage_us": rb["stage_us"],
                         "kernel": STAGE_KERNEL["amr_bubble"], "achieved_GBs": rb["achieved_GBs"],
                         "frac_hbm": rb["achieved_GBs"] / HBM_PEAK_GBS,
                         "adaptation_cycles": {"run": rb["cycles"], "changed_mesh": rb["changed"]}}
    qbs = torch.empty_like(qb)
    dg.dg_rk_stage(mb, ph, 0.0, 1.0, BUBBLE["dt"], qb, qb, qbs)
    qb1 = torch.empty_like(qb)
    f64b = _time_launches(torch, lambda: dg.dg_rk_stage(mb, ph, 0.75, 0.25, BUBBLE["dt"], qb, qbs, qb1), 20)
    mixb = _time_launches(torch, lambda: dg.dg_rk_stage(mb, mixed, 0.75, 0.25, BUBBLE["dt"], qb, qbs, qb1), 20)
    Ra, Rb = torch.empty_like(qb), torch.empty_like(qb)
    dg.dg_rhs(mb, ph, qb, Ra)
    dg.dg_rhs(mb, mixed, qb, Rb)
    out["amr_bubble"]["mixed"] = {"stage_us_fp64": f64b, "stage_us_mixed": mixb, "speedup": f64b / mixb,
                                  "rhs_rel_l2_vs_fp64_library(rho',momentum,Theta')": _field_err(torch, Rb, Ra)}
    lam = torch.randn(qb.shape, dtype=torch.float64, device=qb.device,
                      generator=torch.Generator(qb.device).manual_seed(7))
    g = torch.empty_like(qb)
    rhs_us = _time_launches(torch, lambda: dg.dg_rhs(mb, ph, qb, Ra), 20)
    adj_us = _time_launches(torch, lambda: dg.dg_rhs_adjoint(mb, ph, qb, lam, g), 20)
    out["amr_bubble"]["adjoint_rhs"] = {"rhs_us": rhs_us, "rhs_adjoint_us": adj_us, "ratio": adj_us / rhs_us}
    _progress("extras: AMR warm bubble forced cycle and conservation gap")
    out["amr_bubble"]["forced_cycle"] = forced_cycle(dg, torch, mb, qb)
    # conservation gap at the hanging faces: mortars against pointwise matching, 10
    # SSP-RK3 steps from the same state, change of the rho' and Theta' budgets relative
    # to the total mass (Theta' = rho theta, a tracer with c = theta)
    gap = {}
    for scheme, key in ((dg.DG_NC_MORTAR, "mortar"), (dg.DG_NC_POINTWISE, "pointwise")):
        php = dg.PhysParams(nonconforming=scheme)
        qg, g1, g2 = qb.clone(), torch.empty_like(qb), torch.empty_like(qb)
        b0 = dg.dg_budgets(mb, php, qg)
        for _ in range(10):
            dg.ssp_rk3_step(mb, php, BUBBLE["dt"], qg, g1, g2)
        b1 = dg.dg_budgets(mb, php, qg)
        gap[key] = {"rho_prime_drift_rel_mass": abs(b1[0] - b0[0]) / abs(b0[1]),
                    "theta_prime_drift_rel_mass": abs(b1[2] - b0[2]) / abs(b0[1])}
    out["amr_bubble"]["nonconforming_gap_10_steps"] = gap
    # the same comparison on a passive tracer carried with the Euler state (section 4.2's tracer loss)
    tgap = {}
    for scheme, key in ((dg.DG_NC_MORTAR, "mortar"), (dg.DG_NC_POINTWISE, "pointwise")):
        php = dg.PhysParams(nonconforming=scheme)
        qg, g1, g2 = qb.clone(), torch.empty_like(qb), torch.empty_like(qb)
        c = 1.0 + 0.1 * torch.rand(mb.K, mb.Np, dtype=torch.float64, device=qb.device,
                                   generator=torch.Generator(qb.device).manual_seed(6))
        c1, c2 = torch.empty_like(c), torch.empty_like(c)
        m0 = dg.dg_tracer_mass(mb, c)
        for _ in range(10):
            dg.ssp_rk3_step_tracer(mb, php, BUBBLE["dt"], qg, g1, g2, c, c1, c2)
        tgap[key] = abs(dg.dg_tracer_mass(mb, c) - m0) / abs(m0)
    out["amr_bubble"]["tracer_loss_10_steps_rel"] = tgap
    del qg, g1, g2, lam, g, Ra, Rb, qbs, qb1
    _progress("extras: adjoint configuration")
    from paper_2404_16648_amd import adjoint as adj
    m4 = dg.dg_mesh_build(4, (16, 16, 16), 0, (0.0, 0.0, 0.0), (1000.0, 1000.0, 1000.0))
    q4 = m4.field()
    dg.dg_init_bell(m4, ph, q4, 2.0, (500.0, 500.0, 350.0), (250.0, 250.0, 250.0))
    dt4, n4 = 0.005, 50
    seed = torch.randn(q4.shape, dtype=torch.float64, device=q4.device,
                       generator=torch.Generator(q4.device).manual_seed(3))
    for rep in range(2):  # the first pass loads the kernels; the second is timed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = q4.clone().requires_grad_(True)
        qT = adj.integrate(x, m4, ph, dt4, n4, 10)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        (gx,) = torch.autograd.grad(qT, x, grad_outputs=seed)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    out["adjoint_gradient"] = {"workload": "16^3 hexes, N=4, 50 SSP-RK3 steps (dt=0.005 s), checkpoints every 10",
                               "forward_s": t1 - t0, "backward_s": t2 - t1, "ratio": (t2 - t1) / (t1 - t0)}
    # ---- uniform bubble, 4^3 hexes, N = 4, dt = 0.05 s: launch-bound, reported only
    m1 = dg.dg_mesh_build(4, (4, 4, 4), 0, (0.0, 0.0, 0.0), (1000.0, 1000.0, 1000.0))
    q1c = m1.field()
    dg.dg_init_bell(m1, ph, q1c, 2.0, (500.0, 500.0, 350.0), (250.0, 250.0, 250.0))
    r1, s1, s2, s3 = m1.field(), m1.field(), m1.field(), m1.field()

    def step1():  # the three stage launches of one step, out of place (same state every time)
        dg.dg_rk_stage(m1, ph, 0.0, 1.0, 0.05, q1c, q1c, s1)
        dg.dg_rk_stage(m1, ph, 0.75, 0.25, 0.05, q1c, s1, s2)
        dg.dg_rk_stage(m1, ph, 1.0 / 3.0, 2.0 / 3.0, 0.05, q1c, s2, s3)

    # the configuration's ten steps captured once as a HIP graph and replayed (the
    # launch-bound case: 30 stage launches of ~1 us of work each)
    gs = dg.GraphedSteps(m1, ph, 0.05, q1c.clone(), 10)
    graph_us = _time_launches(torch, gs.replay, 5) / 10.0
    out["uniform_4x4x4_N4"] = {"rhs_us": _time_launches(torch, lambda: dg.dg_rhs(m1, ph, q1c, r1), 20),
                               "step_us": _time_launches(torch, step1, 20),
                               "step_us_hip_graph_of_10_steps": graph_us, "nodes": m1.K * m1.Np}
    _progress("extras: cubed-sphere shell")
    out["sphere_shell"] = sphere_shell(dg, torch)
    _progress("extras: shell transfers")
    out["sphere_shell_transfers"] = shell_transfers(dg, torch)
    _progress("extras: acoustic wave on the shell")
    out["sphere_acoustic_wave"] = (acoustic_wave(dg, torch, hours=args.acoustic_hours) if args.acoustic_hours > 0
                                   else {"skipped": True})
    _progress("extras: refined shell")
    out["sphere_shell_refined"] = sphere_shell_refined(dg, torch)
    _progress("extras: shell with the theta vortex (precision split, adjoint)")
    out["sphere_vortex"] = sphere_vortex(dg, torch)
    _progress("extras: adaptive acoustic wave on the shell")
    out["sphere_acoustic_wave_adaptive"] = (acoustic_wave_adaptive(dg, torch, hours=args.acoustic_hours)
                                            if args.acoustic_hours > 0 else {"skipped": True})
    _progress("extras: long run")
    out["rtb_long_run"] = rtb_long_run(dg, torch, t_end=args.rtb_seconds)
    # ---- measured copy bandwidth (1 GiB device-to-device) beside the 8 TB/s spec
    src = torch.ones(1 << 30, dtype=torch.uint8, device=q.device)
    dst = torch.empty_like(src)
    cu = _time_launches(torch, lambda: dst.copy_(src), 10)
    out["copy_1GiB_GBs"] = 2.0 * (1 << 30) / (cu * 1e-6) / 1e9
    del src, dst
    # ---- measured float64 FMA rate (8 independent chains per thread) beside the 78.6 TF spec
    sink = torch.empty(256 * 4096, dtype=torch.float64, device=q.device)
    flops = dg.dg_fma_burst(4096, 4000, sink)
    fu = _time_launches(torch, lambda: dg.dg_fma_burst(4096, 4000, sink), 5)
    out["fma_f64_TFLOPs"] = flops / (fu * 1e-6) / 1e12
    return out


def cpu_baseline(dg, torch):
    """The oracle on the host cores.  Sample: one Shu-Osher stage (a, b) = (3/4, 1/4)
    of the density current (the headline mesh built by the oracle's own forest from
    its own initial state and flags) from the analytic initial state plus a seeded
    perturbation, as the stage input, with q0 the initial state; timed with 1
    thread and with all the cores this process may use, median of 3 runs each.
    The same stage of the other configurations (uniform 4^3 bubble, AMR warm
    bubble, 16^3 adjoint configuration) with all cores, median of 3.  The library's
    float64 and precision-split stage on the same inputs is compared with the
    oracle's (relative L2 per field)."""
    import numpy as np

    from oracle import euler as eu
    from oracle import forest as fo
    from paper_2404_16648_amd.synth import random_state

    cores = len(os.sched_getaffinity(0))
    nthreads0 = torch.get_num_threads()

    def build(cfg, state_fn, kind):
        """The oracle's initial mesh (its own state and flags) and the flag sequence."""
        desc = fo.ForestDesc(cfg["N"], *cfg["nroot"], cfg["L"], cfg["lo"], cfg["hi"], (0, 0, 0))
        ph = eu.Phys()
        m = fo.build(desc, None)
        seq = []
        for _ in range(cfg["L"]):
            op = eu.Operator(m, ph)
            fl = eu.flags_from_indicator(m, eu.indicator(op, state_fn(op), kind).numpy(), cfg["thr"])
            fl[fl < 0] = 0
            if not (fl > 0).any():
                break
            seq.append(fl)
            m = fo.build(desc, m, fl, fo.PASS_REFINE)
        return m, eu.Operator(m, ph), seq

    def stage_rate(op, q0, qs, reps=3):
        times, out = [], None
        for _ in range(reps):
            t = time.perf_counter()
            out = eu.rk_stage(op, 0.75, 0.25, 0.01, q0, qs)
            times.append(time.perf_counter() - t)
        el = sorted(times)[len(times) // 2]
        return 5 * op.K * (op.N + 1) ** 3 / el, el, out

    def inputs(op, state_fn, seed):
        q0 = state_fn(op)
        pert = torch.as_tensor(random_state(op.K, op.N, seed, (1e-4, 1e-2, 1e-2, 1e-2, 1e-2)))
        return q0, q0 + pert.reshape(q0.shape)

    dc_state = lambda op: eu.density_current_state(op, dtheta=DC["bell"][0])
    m, op, seq = build(DC, dc_state, eu.IND_GRAD_THETA)
    q0, qs = inputs(op, dc_state, 11)
    torch.set_num_threads(1)
    v1, t1, _ = stage_rate(op, q0, qs)
    torch.set_num_threads(cores)
    vall, tall, want = stage_rate(op, q0, qs)
    # the library on the same inputs (float64 and the precision split)
    lm = dg.dg_mesh_build(DC["N"], DC["nroot"], DC["L"], DC["lo"], DC["hi"])
    for fl in seq:  # the oracle's flags replayed on the library's forest
        lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
    same = lm.K == m.K and np.array_equal(lm.tables()["leaf"], np.array(m.leaves, dtype=np.int32).reshape(-1, 5))
    parity = {"same_mesh": bool(same)}
    if same:
        g0 = q0.reshape(5, m.K, -1).contiguous().to("cuda")
        gs = qs.reshape(5, m.K, -1).contiguous().to("cuda")
        w = want.reshape(5, m.K, -1)
        for key, prec in (("fp64", dg.DG_FP64), ("mixed", dg.DG_MIXED)):
            out = torch.empty_like(g0)
            dg.dg_rk_stage(lm, dg.PhysParams(precision=prec), 0.75, 0.25, 0.01, g0, gs, out)
            torch.cuda.synchronize()
            parity[key + "_stage_rel_l2_vs_oracle(rho',momentum,Theta')"] = _field_err(torch, out.cpu(), w)
    del want
    others = {}
    for name, cfg, state_fn, kind in (
            ("uniform_4x4x4_N4", dict(N=4, nroot=(4, 4, 4), L=0, lo=BUBBLE["lo"], hi=BUBBLE["hi"], thr=0.1),
             eu.bubble_state, eu.IND_THETA),
            ("amr_bubble_N7", BUBBLE, eu.bubble_state, eu.IND_THETA),
            ("adjoint_config_16x16x16_N4", dict(N=4, nroot=(16, 16, 16), L=0, lo=BUBBLE["lo"], hi=BUBBLE["hi"],
                                                thr=0.1), eu.bubble_state, eu.IND_THETA)):
        mo, oo, _ = build(cfg, state_fn, kind)
        a0, a1 = inputs(oo, state_fn, 12)
        v, el, _ = stage_rate(oo, a0, a1)
        others[name] = {"value": v, "unit": "DOF-updates/s", "stage_s": el, "leaves": mo.K, "N": mo.N}
    torch.set_num_threads(nthreads0)
    return {"value": vall, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"one SSP-RK3 stage of the density current (K={m.K}, N=4, {m.K * 125} nodes) from the "
                      f"analytic state plus a seeded perturbation, median of 3: {tall:.2f} s on {cores} threads, "
                      f"{t1:.2f} s on 1 thread",
            "value_1_thread": v1, "cpu_model": _cpu_model(), "threads_all": cores,
            "other_configs_all_cores": others, "library_vs_oracle_same_stage": parity}


if __name__ == "__main__":
    main()
