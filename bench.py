#!/usr/bin/env python3
"""Throughput of the D2Q9 BGK + VIBB time step on one MI355X.

One step = one pass of the whole hot path over the lattice: the boundary-link
kernel (velocity-interpolation-based bounce-back for every fluid->solid link and
the momentum-exchange force) and the fused pull-stream / BGK-collision kernel.

Default workload: the random porous medium, 8192 x 2048 nodes, discs of radius
U[5,15] to porosity 0.6, body force 1e-6, tau = 0.7, FP32 storage -- the one
workload whose working set (about 1.2 GB) exceeds the 256 MB last-level cache,
so its bandwidth is an HBM figure.

Prints ONE JSON line: MLUPS over the timed steps (HIP graph replay), the HBM
roofline of the bulk kernel (durations from a separate pass with HIP events
recorded around every launch on the stream the kernels run on), the FP64 CPU
oracle timed on every host core on a bounded sample of the same workload, and the
GPU's error against that oracle run.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SRCS = [os.path.join(ROOT, "paper_1903_01111_amd", "csrc", f)
               for f in ("lbm_step_kernels.h", "lbm_device.h", "lbm_kernels.hip", "lbm_internal.h")]
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "bulk_kernel_porous_8192x2048_f32_counters.txt")
METRIC = ("MLUPS + % HBM roofline at stated drag/velocity error; "
          "FP16-store & adjoint vs FP32")
BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2, "f32w": 4, "f32p": 4}


def kernel_hash():
    """Hash of the step kernels' sources (a counter summary is valid only for it)."""
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:12]


def bulk_kernel_name(kcfg, layout, storage, coll=0):
    """Template name of the periodic forced bulk kernel (the porous workload) that a
    launch configuration runs (None for the fused form); coll 0 BGK, 1 MRT.  With
    bulk_runs the wavefronts take runs of fluid nodes (compact layout only), with
    bulk_runs 2 reading neighbour words."""
    st = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3, "f32w": 4, "f32p": 5}[storage]
    if kcfg.get("bulk_runs"):
        fused = "true" if kcfg["bulk_fused"] else "false"
        nbr = "true" if kcfg["bulk_runs"] == 2 else "false"
        return f"void bulk_run_kernel<{st}, true, {coll}, {fused}, {nbr}>" if layout == "compact" else None
    if kcfg["bulk_fused"]:
        return None
    b = lambda v: "true" if v else "false"
    return (f"void bulk_kernel<{st}, false, true, {kcfg['bulk_block_x']}, {b(kcfg['bulk_store_solid'])}, "
            f"{b(layout == 'compact')}, {max(kcfg.get('bulk_rows', 1), 1)}, {coll}>")


def counter_traffic(layout, kcfg, storage="f32"):
    """HBM bytes per launch of the bulk kernel shape kcfg from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source and
    population layout and holds that shape; else None."""
    if not os.path.exists(COUNTER_SUMMARY):
        return None
    txt = open(COUNTER_SUMMARY).read()
    m = dict(re.findall(r"^(\w+):\s*(\S+)", txt, flags=re.M))
    if m.get("kernel_source_sha256_12") != kernel_hash() or m.get("layout") != layout:
        return None
    name = bulk_kernel_name(kcfg, layout, storage)
    for line in txt.splitlines():
        parts = [p.strip() for p in line[len("variant:"):].split("|")] if line.startswith("variant:") else []
        if len(parts) >= 4 and parts[0] == name:
            try:
                return float(parts[3])
            except ValueError:
                return None
    return None


def workload(name):
    from paper_1903_01111_amd import workloads as W
    if name == "porous":
        return W.porous_medium()
    if name == "cylinder":
        return W.cylinder_channel()
    if name == "dense":
        # the same lattice with no obstacle: every node fluid, no links (bulk kernel only)
        import numpy as np
        c = W.Case("dense_8192x2048", 8192, 2048, False, 0.7, gx=1e-6)
        y = np.arange(2048)[:, None] * np.ones((1, 8192))
        c.init_ux = 1e-3 * np.sin(2 * np.pi * y / 2048)
        return c
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(case, mask, n_links, storage):
    """Bytes the method must move per launch (each input read once, each output
    written once), as the algorithmic count of the step:
    bulk: 9 loads + 9 stores per fluid node and a 1-byte node type per node (the
          implementation reads a 2-byte mask word that also carries the node's link
          directions; those bytes are not counted), plus the two open columns
          written again;
    link: per link 8 bytes of record (node and direction, q), the two populations
          f+_{i'} at x_f and x_ff, 24 bytes of moments (rho, u at x_f and x_ff in
          FP32), and the stored value is counted in the bulk kernel's pull."""
    s = BYTES[storage]
    n = case.nx * case.ny
    nf = int((mask == 0).sum())
    bulk = nf * 18 * s + n
    if case.x_open:
        bulk += 2 * case.ny * 9 * s
    link = n_links * (8 + 2 * s + 24)
    return bulk, link


def timed(B, lat, steps):
    """steps with every launch bracketed by HIP events; (ms total, link ms, bulk ms)."""
    import torch
    B.lbm_set_profiling(lat.ctx, True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    lat.step(steps)
    ev1.record()
    torch.cuda.synchronize()
    link_ms, bulk_ms, n = B.lbm_kernel_times(lat.ctx)
    B.lbm_set_profiling(lat.ctx, False)
    return ev0.elapsed_time(ev1), link_ms, bulk_ms


def replay_then_timed(B, lat, steps, ksteps=200):
    """ms for `steps` steps with graph replay (as the headline), then (link ms,
    bulk ms, steps) from a shorter pass with HIP events around every launch."""
    import torch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    lat.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ksteps = min(steps, ksteps)
    _, link_ms, bulk_ms = timed(B, lat, ksteps)
    return e0.elapsed_time(e1), link_ms, bulk_ms, ksteps


def e_u(a, b):
    import numpy as np
    ref = max(np.abs(b[0]).max(), np.abs(b[1]).max())
    return float(max(np.abs(a[0] - b[0]).max(), np.abs(a[1] - b[1]).max()) / ref)


def oracle_reference(case, steps, threads):
    """The FP64 oracle on the full workload from its initial state: (ux, uy, force
    sum of object 0, seconds, threads used)."""
    import oracle
    g = oracle.case_geometry(case)
    fp = oracle.init_equilibrium(g.solid, *case.init_fields())
    _, used = oracle.threads_for(threads)
    t0 = time.perf_counter()
    fs, _, _ = oracle.run(fp, g, tau=case.tau, gx=case.gx, gy=case.gy, rho0=case.rho0, x_open=case.x_open,
                          n_obj=case.n_obj, nsteps=steps, u_in=case.inlet(), scheme=oracle.case_scheme(case, g),
                          threads=threads, **oracle.case_kwargs(case))
    sec = time.perf_counter() - t0
    _, ux, uy = oracle.moments(fp, g.solid, (case.gx, case.gy), threads=threads)
    del fp
    return ux, uy, fs[0].copy(), sec, used


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model}


def form_precision(B, case, ref, steps_time, layout="compact", steps_long=20000, storages=None):
    """Every storage form against the FP64 oracle on the full workload, from the
    same initial state: velocity error e_u = max|u - u_oracle| / max|u_oracle| and
    drag error after ref["steps"] steps; the 16-bit forms also against FP32 after
    steps_long steps (e_u and the mean u_x, the superficial velocity), FP16 with the
    scale 2^k from the FP32 run's largest deviation after steps_long steps; then
    throughput (graph replay) and the bulk kernel's time and algorithmic bandwidth.
    ref: dict(ux, uy, force, steps) from oracle_reference."""
    import numpy as np
    n = ref["steps"]
    uo, vo, fo = ref["ux"], ref["uy"], ref["force"]
    storages = storages or [("f32", 0), ("f32p", 0), ("f32w", 0), ("f16", None), ("bf16", 0)]
    out = {"reference": f"FP64 oracle, {n} steps of the full lattice from the initial state"}
    long32 = None
    k16 = None
    for st, kk in storages:
        if kk is None:
            kk = k16
        lat = B.Lattice(case, storage=st, dev_scale_log2=kk, layout=layout)
        lat.step(n)
        r = {"steps": n}
        try:
            _, u, v = lat.moments()
            _, fs, _ = lat.force(0)
            r.update(e_u_vs_oracle=e_u((u, v), (uo, vo)),
                     drag_err_vs_oracle=float(abs(fs[0] - fo[0]) / abs(fo[0])))
            if st == "f32":
                lat.step(steps_long - n)
                _, ul, vl = lat.moments()
                long32 = (ul, vl)
                # the FP16 scale from the largest deviation of the developed flow
                k16 = B.dev_scale_for(B.lbm_max_deviation(lat.ctx))
            elif st in ("f16", "bf16") and long32 is not None:
                r["scale_log2"] = kk
                lat.step(steps_long - n)
                _, ul, vl = lat.moments()
                r.update(e_u_vs_f32_long=e_u((ul, vl), long32), steps_long=steps_long,
                         mean_ux_err_vs_f32_long=float(abs(ul.mean() - long32[0].mean()) / abs(long32[0].mean())))
        except B.LbmError as e:
            r["error"] = f"unstable ({e})"
        B.lbm_autotune(lat.ctx, 30)
        ms, link_ms, bulk_ms, ksteps = replay_then_timed(B, lat, steps_time)
        bulk_bytes, _ = algorithmic_bytes(case, lat.mask, lat.n_links, st)
        bulk_us = bulk_ms * 1e3 / ksteps
        r.update(mlups=round(case.nx * case.ny * steps_time / (ms * 1e-3) / 1e6, 1), bulk_us=round(bulk_us, 2),
                 bulk_GBps_algorithmic=round(bulk_bytes / (bulk_us * 1e-6) / 1e9, 1),
                 bulk_frac_of_hbm_peak=round(bulk_bytes / (bulk_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4))
        out[st] = r
        lat.close()
        print(f"[bench] precision {st}: {r}", file=sys.stderr, flush=True)
    return out


def form_mrt_porous(B, threads, steps_oracle=10, steps_time=500, steps_long=2000):
    """The benchmark workload with the paper's MRT collision (Section 2) in FP32 and
    FP16 storage: velocity and drag error against the FP64 MRT oracle after
    steps_oracle steps of the full lattice, FP16 against FP32 after steps_long
    steps, throughput and the bulk kernel's fraction of the HBM roofline."""
    from paper_1903_01111_amd import workloads as W
    case = W.porous_medium()
    case.collision = "mrt"
    ux, uy, force, sec, used = oracle_reference(case, steps_oracle, threads)
    print(f"[bench] MRT oracle: {steps_oracle} steps on {used} threads in {sec:.1f}s", file=sys.stderr, flush=True)
    out = form_precision(B, case, dict(ux=ux, uy=uy, force=force, steps=steps_oracle), steps_time,
                         steps_long=steps_long, storages=[("f32", 0), ("f16", None)])
    out["workload"] = f"{case.name}, MRT (s_e = s_eps = 1.5, s_q = 1.2, s_nu = 1/tau)"
    return out


def form_batched(B, n_inst, steps, warmup, collisions=("bgk", "mrt")):
    """The batched workload (uneven walled-cylinder channels) in one batch, for each
    collision, run to the stated length: throughput, and how many instances are
    still finite at the end; the BGK batch against a loop over single-lattice
    contexts of the same instances."""
    import numpy as np
    import torch
    from paper_1903_01111_amd import workloads as W
    out = {"workload": f"{n_inst} walled-cylinder channels, nx U{{256..1024}}, ny = nx/4, Re U[20,100]",
           "steps": steps}
    for coll in collisions:
        cases = W.batched_cylinders(n_inst)
        for c in cases:
            c.collision = coll
        geoms = [B.case_geometry(c) for c in cases]
        bt = B.Batch(cases, storage="f32", geometries=geoms)
        bt.step(warmup)
        cfg, tuned_ms = B.lbm_batch_autotune(bt.b, 10)  # keeps the fastest configuration, restores the state
        bt.sync()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        bt.step(steps)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        finite = 0
        for i in range(len(cases)):
            try:
                bt.moments(i)
                finite += 1
            except B.LbmError:
                pass
        bt.close()
        n_nodes = sum(c.nx * c.ny for c in cases)
        taus = [c.tau for c in cases]
        r = {"nodes": n_nodes, "mlups": round(n_nodes * steps / (ms * 1e-3) / 1e6, 1),
             "instances_finite_after": finite, "autotuned": cfg.as_dict(),
             "tau_range": [round(min(taus), 4), round(max(taus), 4)]}
        if coll == "bgk":
            lats = [B.Lattice(c, storage="f32", geometry=g) for c, g in zip(cases, geoms)]
            for lat in lats:
                lat.step(warmup)
            torch.cuda.synchronize()
            nloop = min(steps, 300)
            ev0.record()
            for lat in lats:
                lat.step(nloop)
            ev1.record()
            torch.cuda.synchronize()
            ms_loop = ev0.elapsed_time(ev1)
            for lat in lats:
                lat.close()
            r["single_context_loop_mlups"] = round(n_nodes * nloop / (ms_loop * 1e-3) / 1e6, 1)
            r["speedup_vs_loop"] = round(r["mlups"] / r["single_context_loop_mlups"], 2)
        out[coll] = r
        print(f"[bench] batched {coll}: {r}", file=sys.stderr, flush=True)
    return out


def form_single(B, case, steps, warmup, layout="dense"):
    """Throughput with graph replay (as the headline), then the kernel times from a
    shorter pass with HIP events around every launch."""
    lat = B.Lattice(case, storage="f32", layout=layout)
    lat.step(warmup)
    B.lbm_autotune(lat.ctx, 30)
    lat.step(warmup)
    ms, link_ms, bulk_ms, ksteps = replay_then_timed(B, lat, steps)
    lat.moments()
    cfg = B.lbm_get_kernel_config(lat.ctx).as_dict()
    lat.close()
    return {"mlups": round(case.nx * case.ny * steps / (ms * 1e-3) / 1e6, 1),
            "bulk_us": round(bulk_ms * 1e3 / ksteps, 2), "link_us": round(link_ms * 1e3 / ksteps, 2),
            "kernel_config": cfg}


def upward_crossings(t, y):
    """Times at which y crosses zero upwards (linear interpolation between samples)."""
    import numpy as np
    k = np.nonzero((y[:-1] < 0) & (y[1:] >= 0))[0]
    return t[k] + (t[k + 1] - t[k]) * (-y[k]) / (y[k + 1] - y[k])


def form_cylinder_flow(B, steps=100000, window=16, tail=40000, storage="f32"):
    """Flow past the disc of the 2048x512 channel at Re = 100 (uniform inlet U = 0.05,
    R = 20): mean drag coefficient, rms lift coefficient and Strouhal number of
    the vortex shedding over the last `tail` steps, from the force averaged over
    windows of `window` steps.  C_D = 2 F_x / (rho0 U^2 D) and C_L = 2 F_y /
    (rho0 U^2 D) with the momentum-exchange force on the disc; St = f D / U with f
    from the mean spacing of the lift's upward zero crossings."""
    import numpy as np
    from paper_1903_01111_amd import workloads as W
    case = W.cylinder_channel()
    U, D = 0.05, 2.0 * case.prims[0].r
    lat = B.Lattice(case, storage=storage)
    prev = np.zeros(2)
    samples = []
    w0 = time.perf_counter()
    for _ in range(steps // window):
        lat.step(window)
        _, s, _ = lat.force(0)
        samples.append((s - prev) / window)
        prev = s.copy()
    wall = time.perf_counter() - w0
    lat.moments()  # raises on a non-finite state
    lat.close()
    f = np.array(samples)
    nt = tail // window
    t = (np.arange(len(f)) + 0.5) * window
    cd = 2.0 * f[-nt:, 0] / (U * U * D)
    cl = 2.0 * f[-nt:, 1] / (U * U * D)
    up = upward_crossings(t[-nt:], cl - cl.mean())
    st = float(D / U / np.diff(up).mean()) if len(up) >= 2 else None
    return {"workload": f"{case.name}, Re = 100, U = {U}, D = {D:g}", "storage": storage,
            "steps": steps, "tail": tail,
            "window": window, "C_D_mean": round(float(cd.mean()), 4),
            "C_L_rms": round(float(np.sqrt(np.mean((cl - cl.mean()) ** 2))), 4),
            "C_L_mean": round(float(cl.mean()), 5), "St": round(st, 4) if st else None,
            "shedding_periods_in_tail": max(len(up) - 1, 0), "wall_s": round(wall, 2)}


def form_adjoint(B, steps=2000, ckpt=100):
    """Drag gradient of the uniform-inlet cylinder 1024x256 (R = 12.4, Re = 100):
    wall time of the adjoint call (forward sweep with checkpoints, recomputation,
    reverse sweep) against the plain FP32 forward over the same steps, and the
    FP32 gradient dJ/d(U, cx, cy, R) against the FP64 one."""
    import numpy as np
    import torch
    from paper_1903_01111_amd import workloads as W
    from paper_1903_01111_amd.autograd import drag_and_gradient, with_parameters
    base = W.adjoint_cylinder(nsteps=steps)
    p0 = [0.05, base.prims[0].cx, base.prims[0].cy, base.prims[0].r]
    case = with_parameters(base, *p0)
    # plain forward, FP32, same steps from the same initial state
    lat = B.Lattice(case, storage="f32")
    lat.step(64)
    rho, ux, uy = case.init_fields()
    B.lbm_init_equilibrium(lat.ctx, rho, ux, uy)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    lat.step(steps)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1)
    # adjoint call (one short call first loads its kernels)
    B.lbm_init_equilibrium(lat.ctx, rho, ux, uy)
    lat.adjoint_force(2 * ckpt, ckpt)
    B.lbm_init_equilibrium(lat.ctx, rho, ux, uy)
    B.lbm_force_reset(lat.ctx)
    torch.cuda.synchronize()
    e0.record()
    lat.adjoint_force(steps, ckpt)
    e1.record()
    torch.cuda.synchronize()
    adj_ms = e0.elapsed_time(e1)
    ws = B.lbm_adjoint_workspace_bytes(lat.ctx, steps, ckpt)
    lat.close()
    J32, g32 = drag_and_gradient(base, p0, steps, ckpt, "f32")
    J64, g64 = drag_and_gradient(base, p0, steps, ckpt, "f64")
    err = np.abs(g32 - g64) / np.abs(g64)
    return {"workload": f"adjoint_cylinder_{case.nx}x{case.ny}_R{case.prims[0].r}_Re100",
            "steps": steps, "ckpt_every": ckpt, "forward_ms": round(fwd_ms, 2),
            "adjoint_ms": round(adj_ms, 2), "adjoint_over_forward": round(adj_ms / fwd_ms, 2),
            # bytes per fluid node and step against the forward's 18 values: forward sweep
            # 18, recompute 18 (1 - k/n) (the last segment is taped by the sweep), reverse 27
            "algorithmic_ratio": round((18 + 18 * (1 - ckpt / steps) + 27) / 18, 2),
            "workspace_mb": round(ws / 2 ** 20, 1),
            "J_f32": J32, "J_f64": J64, "grad_f32": [float(v) for v in g32],
            "grad_f64": [float(v) for v in g64],
            "grad_rel_err_f32_vs_f64": [float(v) for v in err],
            "params": "(U, cx, cy, R); tau fixed"}


SCHEME_NAMES = {0: "vibb", 1: "hbb", 2: "bouzidi", 3: "yu"}


def _batch_read_at(B, cases, targets, storage="f64", read=None, chunk=None):
    """One batch of the cases; instance i is read by read(bt, i) once the batch
    has run targets[i] steps (rounded up to whole graphs).  Returns the readings
    and the steps run."""
    import numpy as np
    bt = B.Batch(cases, storage=storage)
    order = np.argsort(targets, kind="stable")
    done = 0
    out = [None] * len(cases)
    for i in order:
        t = int(-(-int(targets[i]) // 16) * 16)
        if t > done:
            bt.step(t - done)
            done = t
        out[i] = read(bt, int(i))
    bt.close()
    return out, done


def form_wall_sweep(B, qs=(0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9), res=(6.0, 60.0),
                    taus=(0.51, 0.55, 0.6, 0.7, 0.8, 0.9, 1.0), schemes=(0, 2, 3), storage="f64",
                    decay=4.0):
    """Section 4.1 in one batched launch: Poiseuille flow with a moving top wall
    (L = 60, g = 1e-6, u_top = 0.01, bottom wall halfway bounce-back, top wall at q
    by the scheme under test), MRT collision.  Error vs q at Re = 6 and 60, and vs
    tau at q = 0.8: the paper's |(u_s - u_e)/u_e| after each instance has run
    `decay` slowest-mode decay times from the exact profile.  Reading: the paper
    plots this error against the top wall's q without saying where it is taken;
    it is reported at the boundary node next to the moving wall ("top_node", the
    node the closure acts on) and as its maximum over the fluid rows ("max_rows",
    which the fixed halfway bounce-back bottom wall dominates: with MRT at these
    rates its slip error is the same for every top-wall scheme).  The paper's
    statements about the three schemes are evaluated on the top-node error as
    inequalities and reported, true or false."""
    import numpy as np
    from paper_1903_01111_amd import workloads as W
    cases, tags = [], []
    for re in res:
        for q in qs:
            for s in schemes:
                cases.append(W.moving_wall_poiseuille(q, re, s))
                tags.append(("re", re, q, s))
    for tau in taus:
        for s in schemes:
            cases.append(W.moving_wall_poiseuille(0.8, 0.0, s, tau=tau))
            tags.append(("tau", tau, 0.8, s))
    L, g, ut = 60, 1e-6, 0.01

    def err(bt, i):
        c, tag = cases[i], tags[i]
        q = tag[2]
        nu = (c.tau - 0.5) / 3.0
        yb, H = 0.5, L - 0.5 + q
        _, ux, _ = bt.moments(i)
        y = np.arange(1, L + 1) - yb
        ue = -g / (2 * nu) * y ** 2 + (g * H / (2 * nu) + ut / H) * y
        e = np.abs((ux[1:L + 1, 0] - ue) / ue)
        return float(e[-1]), float(e.max())

    targets = []
    for c, tag in zip(cases, tags):
        nu = (c.tau - 0.5) / 3.0
        H = L - 0.5 + tag[2]
        targets.append(decay * H * H / (np.pi ** 2 * nu))
    t0 = time.perf_counter()
    errs, steps = _batch_read_at(B, cases, targets, storage, err)
    wall = time.perf_counter() - t0
    out = {"workload": "Section 4.1 moving-wall Poiseuille, L = 60, g = 1e-6, u_top = 0.01, MRT, "
                       f"{len(cases)} instances in one batch ({storage})",
           "error": "max over fluid rows of |(u_s - u_e)/u_e| (the paper's metric)",
           "q": list(qs), "tau": list(taus), "steps": steps, "wall_s": round(wall, 2)}
    for m, name in ((0, "top_node"), (1, "max_rows")):
        d = {}
        for re in res:
            d[f"re{re:g}"] = {SCHEME_NAMES[s]: [errs[k][m] for k, tg in enumerate(tags)
                                                if tg[0] == "re" and tg[1] == re and tg[3] == s] for s in schemes}
        d["tau_q0.8"] = {SCHEME_NAMES[s]: [errs[k][m] for k, tg in enumerate(tags) if tg[0] == "tau" and tg[3] == s]
                         for s in schemes}
        out[name] = d
    if set(schemes) >= {0, 2, 3} and 60.0 in res and 6.0 in res:
        hi = [k for k, q in enumerate(qs) if q > 0.5]
        lo = [k for k, q in enumerate(qs) if q < 0.5]
        r60, r6, tt = (out["top_node"][k] for k in ("re60", "re6", "tau_q0.8"))
        best_other60 = [min(r60["bouzidi"][k], r60["yu"][k]) for k in hi]
        spread = {n: max(v) / min(v) for n, v in tt.items()}
        out["paper_statements"] = {
            "re60: VIBB error falls as q grows beyond 1/2":
                all(r60["vibb"][a] >= r60["vibb"][b] for a, b in zip(hi, hi[1:])),
            "re60: VIBB below both other schemes for every q > 1/2":
                all(r60["vibb"][k] < o for k, o in zip(hi, best_other60)),
            "re60: smallest ratio other/VIBB for q > 1/2": round(min(o / r60["vibb"][k]
                                                                      for k, o in zip(hi, best_other60)), 2),
            "re6: VIBB not above the others for q > 1/2":
                all(r6["vibb"][k] <= min(r6["bouzidi"][k], r6["yu"][k]) for k in hi),
            "re6: largest ratio between schemes for q < 1/2": round(max(
                max(r6[a][k] for a in r6) / min(r6[a][k] for a in r6) for k in lo), 2),
            "tau sweep: max/min error over tau per scheme": {n: round(v, 2) for n, v in spread.items()},
            "tau sweep: VIBB depends least on tau": spread["vibb"] < min(spread["bouzidi"], spread["yu"]),
        }
    return out


def _couette_error(ux, uy, solid, case):
    """Relative L2 error of the fluid velocity against Section 4.2's exact profile
    u_theta(r) = u_w R1 (R2/r - r/R2) / (R2/R1 - R1/R2) about the cylinders' centre."""
    import numpy as np
    inner = case.prims[0]
    cx, cy, r1, om = inner.cx, inner.cy, inner.r, inner.omega
    r2 = case.prims[1].r
    L = solid.shape[0]
    yy, xx = np.mgrid[0:L, 0:L]
    dx, dy = xx - cx, yy - cy
    r = np.hypot(dx, dy)
    fl = solid == 0
    ut = om * r1 ** 2 * (r2 ** 2 / r - r) / (r2 ** 2 - r1 ** 2)
    ex, ey = -dy / r * ut, dx / r * ut
    return float(np.sqrt(((ux - ex) ** 2 + (uy - ey) ** 2)[fl].sum() / (ex ** 2 + ey ** 2)[fl].sum()))


def form_couette(B, Ls=(20, 40, 80, 160), res=(6.0, 60.0), res_at_160=(6.0, 12.0, 24.0, 36.0, 48.0, 60.0),
                 schemes=(0, 3), storage="f64", diffusive=1.5):
    """Section 4.2: cylindrical Couette flow, R1 = L/4.8, R2 = L/2.4, L = 20..160 at
    Re = 6 and 60 (Re = u_w L / nu at tau = 0.55, readings), VIBB against Yu's
    scheme, MRT, one batched launch.  Each instance is read after `diffusive` diffusion times
    (R2 - R1)^2 / nu (VIBB and Yu do not conserve mass on curved walls, so there is
    no exact steady state: the start-up transient has then decayed and the drift
    is still negligible).  Error: relative L2 over the fluid nodes; order from
    successive resolutions; the error against Re at L = 160."""
    import numpy as np
    from paper_1903_01111_amd import workloads as W
    cases, tags = [], []
    for re in res:
        for L in Ls:
            for s in schemes:
                cases.append(W.cylindrical_couette(L, re, s))
                tags.append(("L", re, L, s))
    for re in (res_at_160 if 160 in Ls else ()):
        if re in res:
            continue
        for s in schemes:
            cases.append(W.cylindrical_couette(160, re, s))
            tags.append(("L", re, 160, s))
    geoms = [B.case_geometry(c) for c in cases]

    def err(bt, i):
        _, ux, uy = bt.moments(i)
        return _couette_error(ux, uy, geoms[i][0], cases[i])

    targets = [diffusive * (c.prims[1].r - c.prims[0].r) ** 2 / ((c.tau - 0.5) / 3.0) for c in cases]
    t0 = time.perf_counter()
    errs, steps = _batch_read_at(B, cases, targets, storage, err)
    wall = time.perf_counter() - t0
    out = {"workload": f"Section 4.2 cylindrical Couette, MRT, {len(cases)} instances in one batch ({storage})",
           "L": list(Ls), "steps_max": steps, "wall_s": round(wall, 2)}
    for re in res:
        d = {}
        for s in schemes:
            e = [errs[k] for k, tg in enumerate(tags) if tg[1] == re and tg[3] == s and tg[2] in Ls]
            d[SCHEME_NAMES[s]] = {"error": e, "order": [round(float(np.log2(e[k] / e[k + 1])), 3)
                                                         for k in range(len(e) - 1)]}
        out[f"re{re:g}"] = d
    if 160 in Ls:
        res_all = sorted(set(res) | set(res_at_160))
        out["L160_vs_re"] = {"re": res_all, **{SCHEME_NAMES[s]: [
            next(errs[k] for k, tg in enumerate(tags) if tg[1] == re and tg[2] == 160 and tg[3] == s)
            for re in res_all] for s in schemes}}
    if set(schemes) >= {0, 3} and 160 in Ls:
        st = {}
        for re in res:
            v, y = out[f"re{re:g}"]["vibb"], out[f"re{re:g}"]["yu"]
            st[f"re{re:g}: VIBB below Yu at every L"] = all(a < b for a, b in zip(v["error"], y["error"]))
            st[f"re{re:g}: VIBB order, finest pair"] = v["order"][-1]
        ev, ey = out["L160_vs_re"]["vibb"], out["L160_vs_re"]["yu"]
        st["L=160: error grows with Re (VIBB)"] = all(a <= b for a, b in zip(ev, ev[1:]))
        st["L=160: VIBB error at Re 60 over Re 6"] = round(ev[-1] / ev[0], 2)
        st["L=160: Yu error at Re 60 over Re 6"] = round(ey[-1] / ey[0], 2)
        out["paper_statements"] = st
    return out


def form_magnus(B, spins=(0.0, 0.5, 1.0, 1.5, 2.0), steps=40000, window=2000, storage="f64", L=400):
    """Section 4.3: lift on a particle spinning at S_pa = omega R / U in a walled
    Poiseuille channel (L = 400, R = 10, U = 0.05, Re = 2UR/nu = 20), MRT, the
    Galilean-invariant momentum exchange, all spin numbers in one batched launch.
    C_L = F_y / (rho0 U^2 R) and C_D = F_x / (rho0 U^2 R) averaged over the last
    window; the change between the last two windows shows how steady it is.  The
    paper compares with literature values that are not available here: these
    coefficients are parity-unpinned (the kernels match the oracle on the same
    flow at small size in the GPU tests)."""
    import numpy as np
    from paper_1903_01111_amd import workloads as W
    cases = [W.magnus_channel(s, L=L) for s in spins]
    U, R = 0.05, cases[0].prims[0].r
    bt = B.Batch(cases, storage=storage)
    t0 = time.perf_counter()
    bt.step(steps - 2 * window)
    s0 = [bt.force(i, 0)[1].copy() for i in range(len(cases))]
    bt.step(window)
    s1 = [bt.force(i, 0)[1].copy() for i in range(len(cases))]
    bt.step(window)
    s2 = [bt.force(i, 0)[1].copy() for i in range(len(cases))]
    for i in range(len(cases)):
        bt.moments(i)  # finite check
    bt.close()
    wall = time.perf_counter() - t0
    f1 = [(b - a) / window for a, b in zip(s0, s1)]
    f2 = [(b - a) / window for a, b in zip(s1, s2)]
    cl = [float(f[1] / (U * U * R)) for f in f2]
    cd = [float(f[0] / (U * U * R)) for f in f2]
    drift = [float(abs(b[1] - a[1]) / (U * U * R)) for a, b in zip(f1, f2)]
    out = {"workload": f"Section 4.3 Magnus flow, {cases[0].nx}x{cases[0].ny}, R = {R:g}, U = {U}, Re = 20 "
                       f"(nu = {(cases[0].tau - 0.5) / 3:.4g}), MRT, Galilean-invariant momentum exchange, "
                       f"{len(cases)} spin numbers in one batch ({storage})",
           "S_pa": list(spins), "C_L": cl, "C_D": cd, "C_L_change_between_last_windows": drift,
           "steps": steps, "window": window, "wall_s": round(wall, 2),
           "sign": "C_L = F_y/(rho0 U^2 R); a counter-clockwise spin (omega > 0) in a +x stream lifts towards -y"}
    out["checks"] = {"C_L(0) ~ 0 (symmetric channel)": abs(cl[0]) < 1e-3,
                     "|C_L| grows with S_pa": all(abs(a) < abs(b) for a, b in zip(cl, cl[1:])),
                     "C_L < 0 for S_pa > 0": all(c < 0 for c in cl[1:])}
    return out


def form_position(B, n_offsets=64, nx=512, re=20.0, steps=24000, window=2000, storage="f32", schemes=(0, 2, 1)):
    """The solid-position dependency (abstract, Section 5) in one batched launch:
    the walled-cylinder channel at one size and Re with n_offsets sub-grid disc
    offsets, per disc closure (VIBB, Bouzidi, halfway bounce-back; walls halfway
    bounce-back), MRT.  C_D = 2 F_x / (rho0 U_max^2 D) averaged over the last
    window; reported: std(C_D)/mean(C_D) over the offsets for each closure."""
    import numpy as np
    from paper_1903_01111_amd import workloads as W
    cases = W.position_study(n_offsets, nx, re, schemes=schemes)
    D = 2.0 * cases[0].prims[0].r
    U = 0.05
    bt = B.Batch(cases, storage=storage)
    t0 = time.perf_counter()
    bt.step(steps - window)
    a = [bt.force(i, 0)[1].copy() for i in range(len(cases))]
    bt.step(window)
    b = [bt.force(i, 0)[1].copy() for i in range(len(cases))]
    for i in range(len(cases)):
        bt.moments(i)
    bt.close()
    wall = time.perf_counter() - t0
    cd = np.array([2.0 * (y[0] - x[0]) / window / (U * U * D) for x, y in zip(a, b)])
    cl = np.array([2.0 * (y[1] - x[1]) / window / (U * U * D) for x, y in zip(a, b)])
    ns = len(schemes)
    out = {"workload": f"{n_offsets} sub-grid disc offsets x {ns} closures, walled cylinder {nx}x{nx // 4}, "
                       f"Re = {re:g}, R = {cases[0].prims[0].r:g}, MRT, one batch ({storage})",
           "steps": steps, "window": window, "wall_s": round(wall, 2), "nodes": sum(c.nx * c.ny for c in cases)}
    for j, s in enumerate(schemes):
        v, l = cd[j::ns], cl[j::ns]
        out[SCHEME_NAMES[s]] = {"C_D_mean": round(float(v.mean()), 5),
                                "C_D_std_over_mean": float(v.std() / v.mean()),
                                "C_D_range_over_mean": float((v.max() - v.min()) / v.mean()),
                                "C_L_std": float(l.std())}
    if set(schemes) >= {0, 2, 1}:
        out["paper_statement: VIBB depends least on the disc position"] = (
            out["vibb"]["C_D_std_over_mean"] < min(out["bouzidi"]["C_D_std_over_mean"],
                                                   out["hbb"]["C_D_std_over_mean"]))
    return out


DTYPE = {"f64": "f64", "f32": "f32 storage, f32 collision + f64 moments", "f32p": "f32",
         "f32w": "f32 storage, f64 collision", "f16": "f16 storage (x 2^k), f32 arithmetic + f64 moments",
         "bf16": "bf16 storage (x 2^k), f32 arithmetic + f64 moments"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="porous", choices=["porous", "cylinder", "dense"])
    ap.add_argument("--storage", default="f32", choices=list(BYTES))
    ap.add_argument("--layout", default="compact", choices=["dense", "compact"],
                    help="population layout: every node, or the fluid nodes only")
    ap.add_argument("--oracle-steps", type=int, default=100,
                    help="steps of the FP64 oracle on the full lattice, on every host core: the CPU baseline "
                         "and the reference of the stated errors (0: skip)")
    ap.add_argument("--oracle-threads", type=int, default=0, help="oracle threads (0: every core of this process)")
    ap.add_argument("--cpu-single-steps", type=int, default=2,
                    help="steps of the single-thread oracle for its rate (0: skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 1 GiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the storage, batched, cylinder, adjoint and study measurements")
    ap.add_argument("--form", choices=["storage_16bit", "batched", "cylinder", "cylinder_flow", "dense_layout",
                                       "adjoint", "wall_sweep", "couette", "magnus", "position", "mrt_porous"],
                    help="run only this form and print its JSON object")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; a run over several GPUs "
                                   "would split the lattice into y-slabs with halo exchange, "
                                   "which is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1903_01111_amd import binding as B

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    threads = args.oracle_threads or len(os.sched_getaffinity(0))

    def reference(case):
        ux, uy, fs, sec, used = oracle_reference(case, args.oracle_steps, threads)
        print(f"[bench] oracle: {args.oracle_steps} steps on {used} threads in {sec:.1f}s", file=sys.stderr,
              flush=True)
        return {"ux": ux, "uy": uy, "force": fs, "steps": args.oracle_steps, "sec": sec, "threads": used}

    if args.form:
        from paper_1903_01111_amd import workloads as W
        B.lib()
        if args.form == "storage_16bit":
            case = workload(args.workload)
            res = form_precision(B, case, reference(case), 500)
        elif args.form == "batched":
            res = form_batched(B, 256, 10000, 20)
        elif args.form == "cylinder":
            res = form_single(B, W.cylinder_channel(), 2000, 100)
        elif args.form == "cylinder_flow":
            res = form_cylinder_flow(B)
        elif args.form == "dense_layout":
            res = form_single(B, workload(args.workload), 1000, 100, layout="dense")
        elif args.form == "wall_sweep":
            res = form_wall_sweep(B)
        elif args.form == "couette":
            res = form_couette(B)
        elif args.form == "magnus":
            res = form_magnus(B)
        elif args.form == "position":
            res = form_position(B)
        elif args.form == "mrt_porous":
            res = form_mrt_porous(B, threads)
        else:
            res = form_adjoint(B)
        print(json.dumps({"form": args.form, **res}), flush=True)
        return
    t_setup = time.perf_counter()
    case = workload(args.workload)
    lat = B.Lattice(case, storage=args.storage, layout=args.layout)
    n_nodes = case.nx * case.ny
    n_fluid = int((lat.mask == 0).sum())
    nfb = B.lbm_check_geometry(lat.params, lat.mask, lat.node, lat.dir, lat.q, lat.uw, lat.obj,
                               lat.scheme)
    print(f"[bench] {case.name}: {n_nodes} nodes, {n_fluid} fluid, {lat.n_links} links "
          f"({nfb} fall back to halfway bounce-back), storage {args.storage}, "
          f"setup {time.perf_counter() - t_setup:.1f}s", file=sys.stderr, flush=True)

    if args.calibrate_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    lat.step(args.warmup)
    lat.sync()
    cfg, tuned_ms = B.lbm_autotune(lat.ctx, 60)  # keeps the fastest launch shape, restores the state
    print(f"[bench] autotuned {cfg.as_dict()} ({tuned_ms * 1e3:.1f} us/step)", file=sys.stderr,
          flush=True)
    lat.moments()  # raises LBM_E_UNSTABLE on a non-finite state
    lat.step(args.warmup)

    # timed region: graph replay, synchronised on both sides; then the kernel
    # durations from a separate pass with HIP events around every launch on the
    # kernels' stream
    w0 = time.perf_counter()
    ms, link_ms, bulk_ms, ksteps = replay_then_timed(B, lat, args.steps, ksteps=min(args.steps, 200))
    wall = time.perf_counter() - w0
    _, fsum, nsum = lat.force(0)
    lat.moments()  # finite check after the timed steps

    mlups = n_nodes * args.steps / (ms * 1e-3) / 1e6
    bulk_bytes, link_bytes = algorithmic_bytes(case, lat.mask, lat.n_links, args.storage)
    bulk_avg_s = bulk_ms * 1e-3 / ksteps
    link_avg_s = link_ms * 1e-3 / ksteps
    achieved = bulk_bytes / bulk_avg_s / 1e9
    link_gbps = link_bytes / link_avg_s / 1e9 if link_avg_s > 0 else None
    print(f"[bench] {args.steps} steps in {ms:.1f} ms (graph replay): {mlups:.0f} MLUPS; "
          f"bulk {bulk_avg_s * 1e6:.1f} us/launch = {achieved:.0f} GB/s; link "
          f"{link_avg_s * 1e6:.1f} us/launch", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.storage],
        "data": "synthetic",
        "config": {"workload": case.name, "nx": case.nx, "ny": case.ny, "tau": case.tau,
                   "body_force": case.gx, "n_discs": len(case.prims), "fluid_nodes": n_fluid,
                   "links": lat.n_links, "hbb_fallback_links": nfb,
                   "boundary": "VIBB (velocity-interpolation bounce-back)",
                   "collision": "BGK + Guo forcing", "storage": args.storage, "layout": args.layout,
                   "kernel_config": cfg.as_dict(), "timing": "HIP graph replay; kernel durations from a "
                                                             f"separate {ksteps}-step pass with HIP events"},
        "mflups_fluid": round(n_fluid * args.steps / (ms * 1e-3) / 1e6, 1),
        "step_algorithmic_GBps": round((bulk_bytes + link_bytes) / (ms * 1e-3 / args.steps) / 1e9, 1),
        "roofline": {"bound": "hbm", "kernel": "bulk (pull + BGK collision)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counter_traffic(args.layout, cfg.as_dict(), args.storage),
                     "algorithmic_bytes_per_launch": bulk_bytes,
                     "bytes_per_unit": f"18 x {BYTES[args.storage]} B per fluid node + 1 B per node",
                     "avg_launch_us": round(bulk_avg_s * 1e6, 2)},
        "link_kernel": {"avg_launch_us": round(link_avg_s * 1e6, 2),
                        "algorithmic_bytes_per_launch": link_bytes,
                        "bytes_per_unit": f"8 + 2 x {BYTES[args.storage]} + 24 B per link",
                        "GBps": round(link_gbps, 1) if link_gbps and link_gbps <= HBM_PEAK_GBS else None,
                        "frac": round(link_gbps / HBM_PEAK_GBS, 4)
                        if link_gbps and link_gbps <= HBM_PEAK_GBS else None},
        "drag_per_step_mean": [float(fsum[0] / max(nsum, 1)), float(fsum[1] / max(nsum, 1))],
    }

    ref = None
    if args.oracle_steps > 0:
        import oracle

        ref = reference(case)
        rate = n_nodes * args.oracle_steps / ref["sec"] / 1e6
        single = None
        if args.cpu_single_steps > 0:
            g = oracle.case_geometry(case)
            fp = oracle.init_equilibrium(g.solid, *case.init_fields())
            t0 = time.perf_counter()
            oracle.run(fp, g, tau=case.tau, gx=case.gx, gy=case.gy, rho0=case.rho0, x_open=case.x_open,
                       n_obj=case.n_obj, nsteps=args.cpu_single_steps, u_in=case.inlet(),
                       scheme=oracle.case_scheme(case, g), **oracle.case_kwargs(case))
            single = n_nodes * args.cpu_single_steps / (time.perf_counter() - t0) / 1e6
            del fp
        out["cpu_baseline"] = {
            "value": round(rate, 3), "unit": "MLUPS", "cores": ref["threads"], "kind": "oracle",
            "sample": f"{args.oracle_steps} steps of the full {case.nx}x{case.ny} lattice, FP64, OpenMP build of "
                      f"the oracle (bitwise its serial results) on {ref['threads']} threads ({ref['sec']:.1f}s)",
            "single_thread_mlups": round(single, 3) if single else None,
            "single_thread_sample": f"{args.cpu_single_steps} steps, serial build" if single else None,
            "host": host_info()}
        # the headline configuration from the same initial state, same steps
        rho0, ux0, uy0 = case.init_fields()
        B.lbm_init_equilibrium(lat.ctx, rho0, ux0, uy0)
        B.lbm_force_reset(lat.ctx)
        lat.step(args.oracle_steps)
        _, gux, guy = lat.moments()
        _, gfs, _ = lat.force(0)
        out["error_vs_oracle"] = {"e_u": e_u((gux, guy), (ref["ux"], ref["uy"])),
                                  "drag": float(abs(gfs[0] - ref["force"][0]) / abs(ref["force"][0])),
                                  "steps": args.oracle_steps,
                                  "definition": "max|u_gpu - u_oracle| / max|u_oracle|; |F_x - F_x,oracle| / "
                                                "|F_x,oracle| of the force summed over the steps"}
    lat.close()
    if not args.no_forms:
        from paper_1903_01111_amd import workloads as W
        forms = {}
        if ref is not None:
            forms["storage_16bit"] = form_precision(B, case, ref, 500)
            forms["mrt_porous"] = form_mrt_porous(B, threads)
        forms["batched"] = form_batched(B, 256, 10000, 20)
        forms["cylinder_2048x512_f32"] = form_single(B, W.cylinder_channel(), 2000, 100)
        forms["cylinder_2048x512_f32"]["note"] = ("75 MB working set: resident in the 256 MB "
                                                  "last-level cache, not an HBM figure")
        forms["cylinder_flow_re100"] = form_cylinder_flow(B)
        print(f"[bench] cylinder flow: {forms['cylinder_flow_re100']}", file=sys.stderr, flush=True)
        forms["porous_dense_layout_f32"] = form_single(B, case, 1000, 100, layout="dense")
        forms["porous_dense_layout_f32"]["note"] = ("the same porous step with every node of the padded "
                                                    "lattice stored (solid nodes included)")
        forms["adjoint"] = form_adjoint(B)
        for name, fn in (("wall_sweep", form_wall_sweep), ("couette", form_couette), ("magnus", form_magnus),
                         ("position", form_position)):
            forms[name] = fn(B)
            print(f"[bench] {name}: {forms[name].get('paper_statements', forms[name].get('checks'))}",
                  file=sys.stderr, flush=True)
        out["forms"] = forms
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
