#!/usr/bin/env python3
"""Throughput of the GRMHD RK2 step on one MI355X: zone-cycles/s on the 128^3
Kerr-Schild torus (WENO5-Z-AOAH + LLF, FP64), with the roofline of the
dominant kernel and the oracle timed on the host cores.

A step = ghost fill, stage {1,0,1}, con2prim, ghost fill, stage {1/2,1/2,1/2},
con2prim, ghost fill, reductions (the CFL dt of the next step stays on the
device).  Inputs are resident in HBM before the timed region starts.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-cycles/s per GPU, GRMHD RK2 step at 128^3 Kerr-Schild torus; % HBM roofline"
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=128, help="cells per direction of the torus")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--serial", action="store_true",
                    help="torus: every flux launch on the pack's stream (no concurrent directions)")
    ap.add_argument("--fused", action="store_true",
                    help="torus: the optional fused stage (hydro update inside the flux tiles)")
    ap.add_argument("--persist", type=int, default=0,
                    help="persistent flux grid size in workgroups (0, the default: one "
                         "workgroup per tile, which measured faster on every workload)")
    ap.add_argument("--workload", default="torus128",
                    choices=["torus128", "amr640", "mixed192", "fp64_192", "table128", "scalar128",
                             "m1_128", "regrid640"],
                    help="torus128: the headline line (default); amr640: the torus at 256^3 "
                         "effective on ~640 two-level blocks; mixed192 / fp64_192: the torus "
                         "at 192^3 in 27 blocks of 64^3, mixed precision / FP64; table128: "
                         "the 128^3 torus with the synthetic tabulated EOS and the Y_e scalar; "
                         "scalar128: the same with the ideal gas (scalar cost alone); m1_128: "
                         "the implicit gray-M1 collision update of three species on the 128^3 "
                         "torus; regrid640: tag, regrid and remap of the 631-block two-level torus")
    ap.add_argument("--recon", default="weno5z_aoah", choices=list(RECON_NAMES),
                    help="reconstruction of the torus128 workload (default: the headline's)")
    ap.add_argument("--riemann", default="llf", choices=["llf", "hll"],
                    help="Riemann solver of the torus128 workload (default: the headline's)")
    ap.add_argument("--traffic-summary", nargs=4, metavar="CSV",
                    help="write profiles/k_flux_torus128_traffic.json from the rocprofv3 "
                         "counter files of four runs: FETCH_SIZE and WRITE_SIZE of the "
                         "benchmark, then of --copy-calibration")
    ap.add_argument("--trace-summary", metavar="CSV",
                    help="print a markdown table of a rocprofv3 kernel trace (run_kernel_trace.csv): "
                         "per kernel the dispatches, the mean duration over all of them and over "
                         "those that ran alone (overlapping no other dispatch)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (calibrates rocprofv3's "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count)")
    return ap.parse_args()


def copy_calibration():
    """A plain device-to-device copy of exactly 1 GiB, three times."""
    import torch
    n = 1 << 27                                  # float64 elements = 1 GiB
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "copies": 3}), flush=True)


# reconstruction options of the torus workload: name -> (inputs constant name, label)
RECON_NAMES = {"weno5z_aoah": ("RECON_WENO5Z", "WENO5-Z-AOAH"), "mp5": ("RECON_MP5", "MP5"),
               "plm_mc": ("RECON_PLM_MC", "PLM-MC"), "plm_minmod": ("RECON_PLM_MINMOD", "PLM-minmod"),
               "const": ("RECON_CONST", "piecewise constant")}

KERNEL_SOURCES = ("paper_2410_09146_amd/csrc/kernels.h", "paper_2410_09146_amd/csrc/dev.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(faces):
    """HBM bytes per k_flux launch from the committed rocprofv3 counter
    summary, if it was taken on the kernel sources as they are now."""
    path = os.path.join(ROOT, "profiles", "k_flux_torus128_traffic.json")
    if not os.path.exists(path):
        return None
    s = json.load(open(path))
    if s.get("kernel_source_hash") != kernel_source_hash():
        return None
    return s["hbm_bytes_per_launch"]


def flux_faces(n):
    """Faces the main flux tiles of one direction compute on an n^3 block:
    n faces along the direction x (n + 2) x (n + 2) transverse rows."""
    return n * (n + 2) * (n + 2)


def timed_steps(torch, pack, cfl, steps, warmup):
    """(ms eager, ms graph, per-family profile, reductions) of `steps` C-level
    steps after `warmup`, HIP events on the pack's stream."""
    for _ in range(warmup):
        pack.step_c(None, cfl=cfl)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    pack.profile(True)
    torch.cuda.synchronize()
    e0.record(pack.stream)
    for _ in range(steps):
        pack.step_c(None, cfl=cfl)
    e1.record(pack.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = pack.profile_read()
    pack.profile(False)
    red = pack.reductions()
    pack.step_graph(0)
    torch.cuda.synchronize()
    e0.record(pack.stream)
    pack.step_graph(steps)
    e1.record(pack.stream)
    torch.cuda.synchronize()
    return ms, e0.elapsed_time(e1), prof, red


def growth_workload(args, torch, G, I):
    """One JSON line for a growth configuration (not the headline line)."""
    import numpy as np
    if args.workload == "amr640":
        fine = I.torus(n=(256, 256, 256))
        lev, nx, ll = I.amr_layout(fine, target=640, node=32, smallest=16)
        root = I.coarse_problem(fine)
        Ps, Bs = I.mesh_blocks(fine, lev, nx, ll)
        del fine
        pack = G.Pack(root, layout=(nx, ll, lev))
        pack.init_blocks(Ps, Bs)
        del Ps, Bs
        desc = (f"two-level torus, 256^3 effective (level 0 = 128^3, level 1 where rho > 1e-2 "
                f"rho_max): {len(lev)} blocks ({int(sum(lev))} at level 1) of 16^3/32^3/64^3, "
                "FP64, WENO5-Z-AOAH + LLF")
        cfl, prec = root.cfl, "f64"
    elif args.workload in ("table128", "scalar128"):
        prob = I.torus(n=(128, 128, 128))
        tab = I.synthetic_table() if args.workload == "table128" else None
        prob = I.with_ye(prob, I.torus_ye, tab)
        pack = G.Pack(prob)
        pack.init()
        desc = ("torus 128^3 (one block), WENO5-Z-AOAH + LLF, FP64, Y_e passive scalar, " +
                (f"tabulated EOS ({tab.n[0]}x{tab.n[1]}x{tab.n[2]} nodes in ln rho, ln eps, Y_e; "
                 "synthetic)" if tab is not None else "ideal gas"))
        cfl, prec = prob.cfl, "f64"
    else:
        prob = I.torus(n=(192, 192, 192))
        mixed = args.workload == "mixed192"
        pack = G.Pack(prob, nblk=(3, 3, 3), precision=G.PREC_MIXED if mixed else G.PREC_FP64)
        pack.init()
        desc = ("torus 192^3 in 27 blocks of 64^3, WENO5-Z-AOAH + LLF, " +
                ("mixed precision (FP32 staging, reconstruction, Riemann; FP64 state, "
                 "densitization, RK, inversion)" if mixed else "FP64"))
        cfl, prec = prob.cfl, "f32/f64" if mixed else "f64"
    nx = pack.nx
    ncell = int((nx[:, 0] * nx[:, 1] * nx[:, 2]).sum())
    pack.reductions(sync=False)
    tiles, _ = pack.autotune(reps=2)
    pack.set_persistent(args.persist)
    ms, ms_graph, prof, red = timed_steps(torch, pack, cfl, args.steps, args.warmup)
    faces = int(sum(nx[:, 0] * (nx[:, 1] + 2) * (nx[:, 2] + 2)))      # per direction (cubes)
    opc = json.load(open(os.path.join(ROOT, "paper_2410_09146_amd", "opcount", "opcount.json")))
    fams = ("flux_x1", "flux_x2", "flux_x3")
    avg = sum(prof[f][0] for f in fams) / sum(prof[f][1] for f in fams)
    out = {"metric": "zone-cycles/s, GRMHD RK2 step (growth configuration)",
           "value": round(ncell * args.steps / (ms * 1e-3), 1), "unit": "zone-cycles/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms / args.steps, 4), "higher_is_better": True,
           "dtype": prec, "data": "synthetic",
           "config": {"workload": desc, "cells": ncell, "blocks": int(len(nx))},
           "graph_replay": {"ms_per_step": round(ms_graph / args.steps, 4),
                            "value": round(ncell * args.steps / (ms_graph * 1e-3), 1)},
           "k_flux": {"avg_launch_ms": round(avg, 4), "faces_per_launch": faces},
           "kernels": {k: round(v[0] / args.steps, 4) for k, v in prof.items()},
           "tiling": tiles,
           "state": {"dt": red["dt"], "divb_rel": red["divb_rel"], "c2p_fail": red["c2p_fail"],
                     "c2p_fail_total": red["c2p_fail_total"]}}
    if args.workload not in ("table128", "scalar128"):     # the operation count is the ideal path's
        out["k_flux"]["algorithmic_TFLOPs"] = round(
            opc["per_face_flux_ks_weno_llf"] * faces / (avg * 1e-3) / 1e12, 3)
    print(json.dumps(out), flush=True)


def m1_workload(args, torch, G, I):
    """One JSON line for the implicit gray-M1 collision update (three species)
    on the 128^3 torus: each timed launch starts from the same moments (a
    device copy restores them outside the timed kernel)."""
    prob = I.torus(n=(128, 128, 128))
    R, kap = I.m1_fields(prob)
    pack = G.Pack(prob)
    pack.init()
    R0 = torch.from_numpy(pack.to_pack_layout(R).reshape(3, 4, -1)).to(pack.device).contiguous()
    Kd = torch.from_numpy(pack.to_pack_layout(kap).reshape(3, 3, -1)).to(pack.device).contiguous()
    del R, kap
    Rd = R0.clone()
    it = torch.zeros(pack.nct, dtype=torch.uint8, device=pack.device)
    dt = 0.006
    for _ in range(args.warmup):
        Rd.copy_(R0)
        pack.m1_source(Rd, Kd, dt, iters=it)
    pack.profile(True)
    for _ in range(args.steps):
        Rd.copy_(R0)
        pack.m1_source(Rd, Kd, dt, iters=it)
    prof = pack.profile_read()
    ms, cnt = prof["m1"]
    pack._out()
    torch.cuda.synchronize()
    iters = it.cpu().numpy()
    ncell = 128 ** 3
    per = ms / cnt
    bytes_cell = 3 * 4 * 8 * 2 + 3 * 3 * 8 + 3 * 8           # R in/out, opacities, u-tilde
    live = iters[iters > 0]
    out = {"metric": "cell-species implicit M1 updates/s (growth configuration)",
           "value": round(3 * ncell / (per * 1e-3), 1), "unit": "cell-species/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_launch": round(per, 4), "higher_is_better": True, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "implicit gray-M1 collision update, 3 species, on the 128^3 "
                                  "Kerr-Schild torus (dt 0.006, synthetic opacities)",
                      "cells": ncell},
           "hbm_view": {"algorithmic_bytes_per_cell": bytes_cell,
                        "achieved_GBs": round(bytes_cell * ncell / (per * 1e-3) / 1e9, 1),
                        "frac_of_8TBs": round(bytes_cell * ncell / (per * 1e-3) / 8e12, 4)},
           "newton": {"mean_max_over_species": round(float(live.mean()), 3) if live.size else 0.0,
                      "max": int(iters.max()), "failed_cells": int((iters == 255).sum())}}
    print(json.dumps(out), flush=True)


def regrid_workload(args, torch, G, I):
    """One JSON line for a refinement cycle of the 631-block two-level torus:
    tag the blocks by the density indicator, refine the 8 most structured
    level-0 blocks and derefine every complete sibling group of level-1
    blocks whose indicator is below 0.05, remap, fill ghosts, invert."""
    import time
    import numpy as np
    fine = I.torus(n=(256, 256, 256))
    lev, nx, ll = I.amr_layout(fine, target=640, node=32, smallest=16)
    root = I.coarse_problem(fine)
    Ps, Bs = I.mesh_blocks(fine, lev, nx, ll)
    del fine
    pack = G.Pack(root, layout=(nx, ll, lev))
    pack.init_blocks(Ps, Bs)
    del Ps, Bs
    pack.reductions(sync=False)
    pack.step_c(None, cfl=root.cfl)
    r0 = pack.reductions()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ind = pack.tag(0)
    t1 = time.perf_counter()
    coarse = [b for b in np.argsort(ind)[::-1] if lev[b] == 0][:8]
    tags = [1 if b in coarse else (-1 if lev[b] == 1 and ind[b] < 0.05 else 0) for b in range(len(lev))]
    nx2, ll2, lv2 = G.regrid_layout(pack, tags)
    t2 = time.perf_counter()
    new = G.Pack(root, layout=(nx2, ll2, lv2))
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    new.remap_from(pack)
    new._out()
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    r1 = new.reductions()
    cells = int(sum(np.prod(np.reshape(nx2, (-1, 3)), axis=1)))
    out = {"metric": "refinement cycle of the two-level torus (growth configuration)",
           "value": round((t4 - t3) * 1e3, 2), "unit": "ms (remap + ghosts + inversion)",
           "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "two-level torus, 256^3 effective, tag by the density indicator, "
                                  "refine the 8 most structured level-0 blocks, derefine smooth "
                                  "sibling groups", "blocks_before": len(lev), "blocks_after": len(lv2),
                      "cells_after": cells},
           "ms": {"tag": round((t1 - t0) * 1e3, 2), "layout": round((t2 - t1) * 1e3, 2),
                  "new_pack": round((t3 - t2) * 1e3, 2),
                  "remap_ghosts_inversion": round((t4 - t3) * 1e3, 2)},
           "checks": {"divb_rel_after": r1["divb_rel"],
                      "totals_rel_change": float(np.abs(r1["totals"] - r0["totals"]).max()
                                                 / np.abs(r0["totals"]).max()),
                      "floor_hits": r1["floor_hits"], "c2p_fail": r1["c2p_fail"],
                      "refined": int(sum(1 for t in tags if t > 0)),
                      "derefine_tags": int(sum(1 for t in tags if t < 0))}}
    print(json.dumps(out), flush=True)


def traffic_summary(paths):
    """HBM bytes per k_flux launch from rocprofv3 --pmc counter files (KiB per
    dispatch): per direction the production tile shape (the one launched
    most; the autotuner launches every shape a few times), each counter scaled
    by the true bytes of a plain 1 GiB device copy over what the same counter
    reads for it."""
    import collections
    import csv
    import re

    def per_kernel(path, counter):
        acc = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return acc

    fetch, write = per_kernel(paths[0], "FETCH_SIZE"), per_kernel(paths[1], "WRITE_SIZE")
    cf = max(sum(v) / len(v) for v in per_kernel(paths[2], "FETCH_SIZE").values())
    cw = max(sum(v) / len(v) for v in per_kernel(paths[3], "WRITE_SIZE").values())
    copy_bytes = 1 << 30
    ff, wf = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    # the production FP64 WENO5-Z-AOAH + LLF Kerr-Schild tile kernel, unfused
    pat = re.compile(r"void grmhd::k_flux<1, (\d), 2, 0, 1, double, (\d), 0, 0>")
    per_dir = {}
    for counters, key in ((fetch, "fetch"), (write, "write")):
        for name, vals in counters.items():
            m = pat.match(name)
            if not m:
                continue
            d, sh = int(m.group(1)), int(m.group(2))
            cur = per_dir.setdefault(d, {}).get(key)
            if cur is None or len(vals) > cur[2]:
                per_dir[d][key] = (sum(vals) / len(vals), sh, len(vals))
    out_dirs = {}
    for d in sorted(per_dir):
        f, w = per_dir[d]["fetch"], per_dir[d]["write"]
        out_dirs[f"x{d + 1}"] = {"fetch_KiB_raw": round(f[0], 1), "fetch_shape": f[1],
                                 "write_KiB_raw": round(w[0], 1), "write_shape": w[1],
                                 "hbm_bytes": int(f[0] * 1024 * ff + w[0] * 1024 * wf)}
    faces = flux_faces(128)
    cmd = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 150 rocprofv3 --pmc {c} -d "
           "<out>/{d} -o run --output-format csv -- python3 <repo>/bench.py {a}")
    summary = {
        "kernel": "k_flux (FP64, WENO5-Z-AOAH + LLF, Kerr-Schild), 128^3 torus",
        "kernel_source_hash": kernel_source_hash(),
        "hbm_bytes_per_launch": int(sum(v["hbm_bytes"] for v in out_dirs.values()) / len(out_dirs)),
        "algorithmic_bytes_per_launch": faces * 120,
        "calibration": {"copy_bytes": copy_bytes, "FETCH_SIZE_KiB": round(cf, 1),
                        "WRITE_SIZE_KiB": round(cw, 1), "fetch_factor": round(ff, 5),
                        "write_factor": round(wf, 5)},
        "per_direction": out_dirs,
        "commands": [cmd.format(c="FETCH_SIZE", d="pmc_flux_fetch", a="--steps 2 --warmup 1 --no-cpu-baseline"),
                     cmd.format(c="WRITE_SIZE", d="pmc_flux_write", a="--steps 2 --warmup 1 --no-cpu-baseline"),
                     cmd.format(c="FETCH_SIZE", d="pmc_copy_fetch", a="--copy-calibration"),
                     cmd.format(c="WRITE_SIZE", d="pmc_copy_write", a="--copy-calibration"),
                     "python3 bench.py --traffic-summary <the four run_counter_collection.csv files>",
                     "(<repo>: the repository root; <out>: any output directory)"],
        "note": "FETCH_SIZE and WRITE_SIZE are KiB per dispatch, averaged over the dispatches of "
                "the production tile shape of each direction and scaled by the ratio of a plain "
                "1 GiB device copy's true bytes to what the same counter reads for it; "
                "hbm_bytes_per_launch is the mean over the three directions; algorithmic bytes: "
                "64 B read (P 40, the two transverse cell-centred B 16, the face B 8) and 56 B "
                "written (7 fluxes) per face"}
    path = os.path.join(ROOT, "profiles", "k_flux_torus128_traffic.json")
    with open(path, "w") as fh:
        json.dump(summary, fh, indent=1)
    print(json.dumps(summary), flush=True)


def trace_summary(path):
    """Per kernel of a rocprofv3 kernel trace: dispatches, mean duration, and
    the mean over the dispatches that overlapped no other one (with the flux
    directions on streams of their own, the graph-replayed steps run them side
    by side, which stretches each; the eager pass that bench.py times kernel by
    kernel runs every launch alone)."""
    import collections
    import csv
    rows = [(r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
            for r in csv.DictReader(open(path))]
    rows.sort(key=lambda r: r[1])
    alone = [True] * len(rows)
    end_max, arg = -1, -1
    for k, (_, t0, t1) in enumerate(rows):
        if t0 < end_max:
            alone[k] = False
            alone[arg] = False
        if t1 > end_max:
            end_max, arg = t1, k
    acc = collections.defaultdict(lambda: [0, 0.0, 0, 0.0, 1e30, 0.0])
    for k, (name, t0, t1) in enumerate(rows):
        a = acc[name]
        d = (t1 - t0) * 1e-3
        a[0] += 1; a[1] += d; a[4] = min(a[4], d); a[5] = max(a[5], d)
        if alone[k]:
            a[2] += 1; a[3] += d
    total = sum(a[1] for a in acc.values())
    print("| kernel | dispatches | mean us | alone: dispatches | alone: mean us | min us | max us | share of summed time |")
    print("|---|---|---|---|---|---|---|---|")
    for name, a in sorted(acc.items(), key=lambda kv: -kv[1][1]):
        if a[1] < 0.002 * total:
            continue
        nm = name.split("(")[0]
        am = f"{a[3] / a[2]:.1f}" if a[2] else "-"
        print(f"| `{nm}` | {a[0]} | {a[1] / a[0]:.1f} | {a[2]} | {am} | {a[4]:.1f} | {a[5]:.1f} | "
              f"{100 * a[1] / total:.1f} % |")


def main():
    args = parse()
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.traffic_summary:
        traffic_summary(args.traffic_summary)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py: the GRMHD step runs on one GPU (asked for {args.gpus}); "
              "no code path here spans a second GPU", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one GPU only; refusing a multi-rank launch", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2410_09146_amd import grmhd as G
    from paper_2410_09146_amd import inputs as I

    if args.workload == "m1_128":
        return m1_workload(args, torch, G, I)
    if args.workload == "regrid640":
        return regrid_workload(args, torch, G, I)
    if args.workload != "torus128":
        return growth_workload(args, torch, G, I)

    n = args.n
    headline = args.recon == "weno5z_aoah" and args.riemann == "llf"
    prob = I.torus(n=(n, n, n), recon=getattr(I, RECON_NAMES[args.recon][0]),
                   riemann=I.RIEMANN_LLF if args.riemann == "llf" else I.RIEMANN_HLL)
    pack = G.Pack(prob, device="cuda:0")
    if args.fused:
        pack.set_fused(True)
    if args.serial:
        pack.set_concurrency(False)
    pack.init()
    pack.reductions(sync=False)        # device-resident dt for the first step
    tiles, tune_ms = pack.autotune(reps=3) if not args.no_autotune else ([0, 0, 0], None)
    if args.persist:
        pack.set_persistent(args.persist)
    stream = pack.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    # the timed steps: the SSPRK2 step captured once into a HIP graph (dt
    # stays on the device) and replayed; warm-up replays first
    for _ in range(args.warmup):
        pack.step_c(None, cfl=prob.cfl)
    pack.step_graph(0)
    pack.step_graph(args.warmup)
    torch.cuda.synchronize()
    e0.record(stream)
    pack.step_graph(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1)

    # the same steps launched one by one from the host, with an event pair
    # around every kernel family (the per-kernel times and the roofline)
    pack.profile(True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        pack.step_c(None, cfl=prob.cfl)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = pack.profile_read()
    pack.profile(False)
    red = pack.reductions()

    ncell = n ** 3
    value = ncell * args.steps / (ms_graph * 1e-3)

    # dominant kernel: the face-flux tile kernel k_flux (one launch per
    # direction and stage; the three directions are one template); roofline
    # from algorithmic FP64 flops per face
    opc = json.load(open(os.path.join(ROOT, "paper_2410_09146_amd", "opcount", "opcount.json")))
    per_face = opc[f"per_face_flux_ks_{args.recon}_{args.riemann}"]
    fams = ("flux_x1", "flux_x2", "flux_x3")
    t_ms = sum(prof[f][0] for f in fams)
    cnt = sum(prof[f][1] for f in fams)
    avg_ms = t_ms / cnt
    flops = per_face * flux_faces(n)
    achieved = flops / (avg_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
            "traffic": measured_traffic(flux_faces(n)) if headline else None,
            "kernel": "k_flux (x1, x2, x3 launches)",
            "avg_launch_ms": round(avg_ms, 4), "flops_per_face": per_face,
            "faces_per_launch": flux_faces(n),
            "share_of_step": round(t_ms / args.steps / (ms / args.steps), 3)}
    # HBM view of the whole step: 480 algorithmic bytes per zone-cycle
    hbm = {"algorithmic_bytes_per_zone_cycle": 480,
           "achieved_GBs": round(480 * value / 1e9, 1),
           "frac_of_8TBs": round(480 * value / 1e9 / HBM_PEAK_GBS, 4)}
    # the whole step against both roofs: the target is 60 % of the HBM roof,
    # and the step's FP64 work (flux tiles and update by their operation
    # counts; the inversion, whose cost depends on its iterations, not counted)
    step_flops = 2 * (3 * per_face * flux_faces(n) + opc["per_cell_update_ks"] * ncell)
    step_tf = step_flops * args.steps / (ms_graph * 1e-3) / 1e12
    roof["step"] = {"hbm_frac": hbm["frac_of_8TBs"], "hbm_target_frac": 0.6,
                    "hbm_gap_x": round(0.6 / hbm["frac_of_8TBs"], 2),
                    "fp64_flops_per_step": step_flops, "fp64_TFLOPs": round(step_tf, 3),
                    "fp64_frac": round(step_tf / FP64_PEAK_TFLOPS, 4)}

    kernels = {k: {"ms_per_step": round(v[0] / args.steps, 4), "launches_per_step": v[1] / args.steps}
               for k, v in prof.items()}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
        sim = oracle.Sim(prob, nthreads=threads)
        dt0 = sim.dt()
        t0 = time.perf_counter()
        for _ in range(args.cpu_steps):
            sim.step(dt0)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": round(ncell * args.cpu_steps / t_cpu, 1), "unit": "zone-cycles/s",
               "cores": threads, "kind": "oracle",
               "sample": f"{args.cpu_steps} SSPRK2 step(s) of the same {n}^3 torus, "
                         f"{t_cpu:.1f} s wall, {threads} OpenMP threads"}
        # one thread, on a slab of the same torus (same r-theta grid, 8 phi cells)
        slab = I.torus(n=(n, n, 8))
        sim1 = oracle.Sim(slab, nthreads=1)
        dt1 = sim1.dt()
        t0 = time.perf_counter()
        sim1.step(dt1)
        t1 = time.perf_counter() - t0
        cpu["single_thread"] = {"value": round(n * n * 8 / t1, 1), "cores": 1,
                                "sample": f"1 SSPRK2 step of the torus at {n}x{n}x8, {t1:.1f} s wall"}

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "zone-cycles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_graph / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"Kerr-Schild torus {n}^3 (a=0.9375, FM r_in=6 r_max=12, "
                               "gamma=13/9, beta=100 loop field, noise 4e-2 seed 1), "
                               f"{RECON_NAMES[args.recon][1]} + {args.riemann.upper()}, CT, "
                               "SSPRK2, FP64, one meshblock"
                               + (", fused stage" if args.fused else ""),
                   "cells": ncell, "parallelism": "single GPU"},
        "roofline": roof, "hbm_view": hbm, "kernels": kernels,
        "timing": "value and ms_per_step: K graph-replayed steps (the whole SSPRK2 step "
                  "captured once, dt on the device); eager: the same K steps launched from "
                  "the host with an event pair around every kernel family",
        "eager": {"ms_per_step": round(ms / args.steps, 4),
                  "value": round(ncell * args.steps / (ms * 1e-3), 1)},
        "tiling": {"shape_per_direction": tiles,
                   "autotune_ms": None if tune_ms is None else tune_ms.round(4).tolist()},
        "state": {"dt": red["dt"], "divb_rel": red["divb_rel"], "c2p_fail": red["c2p_fail"],
                  "c2p_fail_total": red["c2p_fail_total"],
                  "floor_hits": red["floor_hits"], "c2p_iter_mean": red["c2p_iter_mean"],
                  "c2p_iter_wavemax_mean": red["c2p_iter_wavemax_mean"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
