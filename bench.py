#!/usr/bin/env python
"""Throughput of the HSC / HSC-extension solve on one MI355X.

Workload: the 32^3 cube (32,768 sites, 7-point, t = -1, on-site U[-0.5, 0.5]
seed 0, per-site 1D leads on the x faces), 256 energies uniform in [-6, 6],
eta = 1e-8, kT = 0.025, mu_L/R = +-0.1.  Cluster tree: 3D nested dissection
with planar separators, leaves <= 8 sites per side.  The fold and the
extraction run in double-double (precision 2 and 3: the settings whose results
agree with the oracle to 1e-10 at every energy of the grid, out of the lead
band included); with precision 3, the default, every double-double block
product of depth >= 32 is formed from 8-bit slices on the integer matrix
cores.

One step = diag G^r, diag G^< and T for one batch of energies (16 by default),
inputs resident on the device; consecutive steps walk the 256-point grid in
order, so 16 steps solve every grid energy once.  Besides the timed steps the
line reports: one-energy-per-launch-sequence ("plain") throughput over a few
energies, the error against stored oracle values at 8 of the 256 energies
(tests/golden), the algorithmic roofline of the dominant kernel (HIP events
around every launch of one step), and the CPU oracle (slab RGF) timed on the
host.  Opt-in studies: --alt (the complex128 path on the FP64 matrix cores),
--trilayer, --uneven, --learned-grid.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
# FP64 vector issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one add, multiply or fused
# multiply-add per lane and clock (the published 78.6 TFLOP/s counts an FMA as two flops)
FP64_VALU_PEAK_TOPS = 39.3
# FP64 vector operations of one complex double-double multiply-add in k_dd_gemm (three real products,
# Gauss form, each 1 mul + 3 fma accumulated with a 6-operation two-sum and 2 adds), per flop of the
# 8 M N K complex count
DD_OPS_PER_CMAC = 36
DD_OPS_PER_CFLOP = DD_OPS_PER_CMAC / 8
# dense int8 matrix-core peak of the chip (5.0 P int8 ops/s) and the int8 operations of one complex
# double-double multiply-add in k_oz_gemm: 3 real products (Gauss) x S (S + 1) / 2 slice pairs
# (s + t <= S - 1) x 2; S = 16 slices per operand unless --slices 15
INT8_MFMA_PEAK_TOPS = 5000.0
OZ_DEFAULT_SLICES = 16


def oz_int8_ops_per_cmac(slices):
    s = slices or OZ_DEFAULT_SLICES
    return 3 * (s * (s + 1) // 2) * 2


# HBM traffic of k_oz_gemm per launch from two rocprofv3 --pmc passes over the same workload (the
# benchmark cube, one set-up batch and one step of 16 energies, through the native driver
# paper_1702_05167_amd/hsc_run; profiles/k_oz_gemm_cube32_nd8_counters.md), each scaled by what the
# counter reads for a plain copy of 64 MiB (FETCH_SIZE 32781.3 KiB for 65536 KiB read, WRITE_SIZE
# 65536 KiB for 65536 KiB written).  Valid only for the kernel source and slice count they were
# taken on.
OZ_TRAFFIC = {"sources": ["paper_1702_05167_amd/csrc/ozaki.hip", "paper_1702_05167_amd/csrc/kern.h"],
              "sha256": "593ccb11464d5d8e0e8d93acd64e3e56a31e5f11cb9ab49fbf1c6df4caa12a5c",
              "fetch_kib_per_launch": 2763533.9, "write_kib_per_launch": 1455739.6, "launches": 268,
              "fetch_scale": 65536.0 / 32781.25, "write_scale": 65536.0 / 65536.0}


def oz_sources_sha256():
    """SHA-256 over what defines k_oz_gemm: the slice-product section of ozaki.hip (its staging, matrix-core
    loop, epilogue sums and the kernel) and the slice-count lines of kern.h."""
    import hashlib
    h = hashlib.sha256()
    for rel in OZ_TRAFFIC["sources"]:
        path = os.path.join(ROOT, rel)
        if not os.path.exists(path):
            return None
        data = open(path, "rb").read()
        if rel.endswith("kern.h"):
            data = b"".join(line for line in data.splitlines(keepends=True) if b"constexpr int kOzSlices" in line)
        else:
            a, b = data.find(b"// products of the slices"), data.find(b"// the allocation-free product")
            if a < 0 or b < a:
                return None
            data = data[a:b]
        h.update(data)
    return h.hexdigest()


def oz_traffic():
    """Measured bytes per k_oz_gemm launch, or None when the kernel sources changed since."""
    if oz_sources_sha256() != OZ_TRAFFIC["sha256"]:
        return None
    return 1024.0 * (OZ_TRAFFIC["fetch_kib_per_launch"] * OZ_TRAFFIC["fetch_scale"] +
                     OZ_TRAFFIC["write_kib_per_launch"] * OZ_TRAFFIC["write_scale"])


def note(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def golden_errors(np, gold, gr_all, gl_all, tr_all):
    """max relative error of diag G^r, Im diag G^< (sampled sites) and T at the stored energies;
    row k of the arrays belongs to the k-th stored energy"""
    sites = np.array(gold["sites"])
    ref_gr = np.array(gold["gr_re"]) + 1j * np.array(gold["gr_im"])
    ref_gl = np.array(gold["gl_im"])
    errs = []
    for k in range(len(gold["energies"])):
        gr, gl, tr = gr_all[k][sites], gl_all[k][sites].imag, tr_all[k]
        errs.append(max(np.abs(gr - ref_gr[k]).max() / np.abs(ref_gr[k]).max(),
                        np.abs(gl - ref_gl[k]).max() / np.abs(ref_gl[k]).max(),
                        abs(tr - gold["trans"][k]) / max(gold["trans"][k], 1e-12)))
    band = [abs(e) < 2.0 for e in gold["energies"]]
    return {"energies": gold["energies"], "max_rel_err": errs, "max": max(errs),
            "in_band_max": max(x for x, b in zip(errs, band) if b),
            "out_of_band_max": max(x for x, b in zip(errs, band) if not b)}


def roofline_of(prof, precision, prof_bytes=None, slices=0):
    """Algorithmic roofline of the dominant block-product kernel from per-kind launch timing
    (HIP events on the solver's stream): achieved = sum of 8 M N K over its launches / sum of
    their durations, against the FP64 matrix-core peak."""
    total_ms = sum(v["ms"] for v in prof.values())
    g, gd, go = prof["gemm"], prof["dd_gemm"], prof["oz_gemm"]
    if go["ms"] > max(gd["ms"], g["ms"]):
        ach = go["flops"] / (go["ms"] * 1e-3) / 1e12
        i8 = ach * oz_int8_ops_per_cmac(slices) / 8
        alg_bytes = prof_bytes["oz_gemm"] / go["launches"] if prof_bytes and go["launches"] else None
        # the counters were taken with the default slice count
        traffic = oz_traffic() if (slices or OZ_DEFAULT_SLICES) == OZ_DEFAULT_SLICES else None
        return {"bound": "mfma", "kernel": "k_oz_gemm (complex double-double products from 8-bit slices, "
                                           "integer matrix cores)",
                "achieved": ach, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_MFMA_PEAK_TFLOPS,
                "traffic": traffic, "flop_count": "8 M N K per complex product (algorithmic)",
                "algorithmic_bytes_per_launch": alg_bytes,
                "traffic_over_algorithmic": traffic / alg_bytes if traffic and alg_bytes else None,
                "launches": int(go["launches"]), "avg_launch_ms": go["ms"] / go["launches"],
                "flops_per_launch": go["flops"] / go["launches"],
                "share_of_kernel_time": go["ms"] / total_ms,
                "int8_matrix_cores": {"achieved": i8, "peak": INT8_MFMA_PEAK_TOPS, "unit": "T int8 ops/s",
                                      "frac": i8 / INT8_MFMA_PEAK_TOPS,
                                      "int8_ops_per_complex_multiply_add": oz_int8_ops_per_cmac(slices),
                                      "note": "unpadded M N K; padding to 32 x 32 x 64 tiles not counted"}}
    if precision >= 1 and gd["ms"] > 0:
        ach = gd["flops"] / (gd["ms"] * 1e-3) / 1e12
        issue = DD_OPS_PER_CFLOP * ach
        return {"bound": "alu", "kernel": "k_dd_gemm (grouped complex double-double GEMM, FP64 vector units)",
                "achieved": ach, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_MFMA_PEAK_TFLOPS,
                "traffic": None, "flop_count": "8 M N K per complex product (algorithmic)",
                "launches": int(gd["launches"]), "avg_launch_ms": gd["ms"] / gd["launches"],
                "flops_per_launch": gd["flops"] / gd["launches"],
                "share_of_kernel_time": gd["ms"] / total_ms,
                "fp64_vector_issue": {"achieved": issue, "peak": FP64_VALU_PEAK_TOPS,
                                      "unit": "T FP64 operations/s", "frac": issue / FP64_VALU_PEAK_TOPS,
                                      "fp64_ops_per_complex_multiply_add": DD_OPS_PER_CMAC}}
    ach = g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else 0.0
    return {"bound": "mfma", "kernel": "k_zgemm (grouped complex128 GEMM, all tile shapes)",
            "achieved": ach, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_MFMA_PEAK_TFLOPS,
            "traffic": None, "flop_count": "8 M N K per complex product (algorithmic)",
            "launches": int(g["launches"]),
            "avg_launch_ms": g["ms"] / g["launches"] if g["launches"] else None,
            "flops_per_launch": g["flops"] / g["launches"] if g["launches"] else None,
            "share_of_kernel_time": g["ms"] / total_ms if total_ms else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16, help="timed steps (one energy batch each)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-side", type=int, default=32)
    ap.add_argument("--energies", type=int, default=256, help="points of the energy grid the steps walk")
    ap.add_argument("--batch", type=int, default=16, help="energies per step (one launch sequence)")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-energy-per-launch-sequence run")
    ap.add_argument("--plain-energies", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-single", type=int, default=1,
                    help="also time the oracle on one thread over this many energies (0: skip)")
    ap.add_argument("--no-golden", action="store_true", help="skip the error against stored oracle values")
    ap.add_argument("--precision", type=int, default=3,
                    help="3 (default): fold and extraction in double-double, block products of depth >= 32 from "
                         "8-bit slices on the integer matrix cores; 2: the same on the FP64 vector units; "
                         "1: double-double fold only; 0: complex128 as in Algorithms 1 and 2")
    ap.add_argument("--leaf", type=int, default=8)
    ap.add_argument("--transverse", action="store_true",
                    help="never cut the transport axis (clusters span contact to contact)")
    ap.add_argument("--tune", type=int, default=1, help="1 (default): autotune the GEMM tile shape per launch")
    ap.add_argument("--slices", type=int, default=0,
                    help="8-bit slices per operand of the precision-3 products: 0 (the library's 16) or 15")
    ap.add_argument("--complex3m", type=int, default=1,
                    help="1 (default): three real products per complex multiply-add in every complex128 block "
                         "product; 0: four")
    ap.add_argument("--alt", action="store_true",
                    help="also run the complex128 path on the matrix cores (one step each on the transverse "
                         "leaf-4 tree and on this tree)")
    ap.add_argument("--uneven", type=int, default=0, metavar="D",
                    help="measure D of the 64 uneven cuboids instead: forest batch vs one device at a time")
    ap.add_argument("--uneven-energies", type=int, default=32)
    ap.add_argument("--config2-full", action="store_true",
                    help="all 64 uneven cuboids x 128 energies at --precision on 3D trees (leaves <= 8), "
                         "through hsc_solve_batch four devices at a time, one progress line per call")
    ap.add_argument("--trilayer", action="store_true",
                    help="measure the 40,020-site trilayer x 512 energies instead, with its error")
    ap.add_argument("--learned-grid", action="store_true",
                    help="measure the learned energy grid instead (surrogate training + charge on 3 devices)")
    ap.add_argument("--guard-study", action="store_true",
                    help="measure the complex128 solve with the growth guard instead (256 energies in chunks of 32, "
                         "3D tree, leaf 8, tau 100), with its error at the stored energies")
    ap.add_argument("--dense-steps", type=int, default=2,
                    help="timed steps of the same cube with whole-face contacts (dense self-energy); 0 skips")
    ap.add_argument("--dense-study", action="store_true",
                    help="time per energy with whole-face (dense) and per-site (diagonal) contacts: cubes N^3 and "
                         "elongated Nx x 16 x 16 devices")
    ap.add_argument("--orbital-study", action="store_true",
                    help="time per energy of 10-orbital wires (4 x 4 and 6 x 6 sites across, lengths 32 .. 128)")
    ap.add_argument("--streams-study", action="store_true",
                    help="energies/s of the benchmark cube with concurrent batches: batch 16 on one stream, batch 8 "
                         "on two streams, batch 4 on four (64 energies of the grid each, after one untimed pass)")
    ap.add_argument("--scf-quick", action="store_true",
                    help="with --scf-study: skip the runs to a residual of 1e-8 (for profiling)")
    ap.add_argument("--scf-study", action="store_true",
                    help="time the self-consistent NEGF-Poisson loop on the --n-side cube (64 energies, 4 iterations)")
    ap.add_argument("--write-device", metavar="PATH",
                    help="write the benchmark cube (--n-side) and its energy grid (--energies) as a device file "
                         "for the native driver paper_1702_05167_amd/hsc_run, then exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run one elementwise device copy of MIB MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); energies shard across GPUs "
              "with no communication but the output gather, so the one-GPU figure is the per-GPU rate.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import synth
    if args.write_device:
        write_device(np, synth.config1_device(n_side=args.n_side), np.linspace(-6.0, 6.0, args.energies),
                     args.write_device)
        return
    import torch
    import paper_1702_05167_amd as pkg

    if args.learned_grid:
        learned_grid_study(pkg, synth, np)
        return
    if args.config2_full:
        config2_full(pkg, synth, np, torch, args)
        return
    if args.uneven > 0:
        uneven_study(pkg, synth, np, torch, args)
        return
    if args.trilayer:
        trilayer_study(pkg, synth, np, torch, args)
        return
    if args.guard_study:
        guard_study(pkg, synth, np, torch, args)
        return
    if args.dense_study:
        dense_study(pkg, synth, np, torch, args)
        return
    if args.orbital_study:
        orbital_study(pkg, synth, np, torch, args)
        return
    if args.scf_study:
        scf_study(pkg, synth, np, torch, args)
        return
    if args.streams_study:
        streams_study(pkg, synth, np, torch, args)
        return

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * 131072, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        note(f"copy calibration: {args.calibrate_copy} MiB read + written")

    N, NE, B = args.n_side, args.energies, args.batch
    if B < 1 or B > NE:
        sys.exit("--batch must be in [1, --energies]")
    dev = synth.config1_device(n_side=N)
    tree = pkg.Tree.from_device(dev, leaf_side=args.leaf, transverse=args.transverse)
    st = tree.stats()
    ctx = pkg.Context(0)
    # the grid as numpy builds it (torch.linspace differs from it by an ulp at some points)
    grid = np.linspace(-6.0, 6.0, NE)
    E = torch.tensor(grid, dtype=torch.float64, device="cuda:0")
    kw = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, precision=args.precision, slices=args.slices,
              complex3m=args.complex3m,
              tune=args.tune, batch=B)
    want = pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS
    gpath = os.path.join(ROOT, "tests", "golden", "cube32_sampled.json")
    gold = json.load(open(gpath)) if (N == 32 and NE == 256 and os.path.exists(gpath)) else None

    def batch_of(k):
        # energies of step k: the next B points of the grid, wrapping around
        idx = [(k * B + j) % NE for j in range(B)]
        return E[idx] if idx[0] + B > NE else E[idx[0]: idx[0] + B]

    t_setup = time.perf_counter()
    out = pkg.solve(ctx, tree, batch_of(0), want=want, **kw)     # buffers, plan, tile tuning
    note(f"set-up (plan, tile tuning, first batch): {time.perf_counter() - t_setup:.1f} s")
    for k in range(args.warmup):
        pkg.solve(ctx, tree, batch_of(k), want=want, out=out, sync=False, **kw)
    torch.cuda.synchronize()
    note("warmup done")
    ok = True
    t0 = time.perf_counter()
    for k in range(args.steps):
        pkg.solve(ctx, tree, batch_of(k), want=want, out=out, sync=False, **kw)
        if (k + 1) % 4 == 0 or k + 1 == args.steps:
            torch.cuda.synchronize()
            note(f"step {k + 1} of {args.steps} done")
    ctx.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = int(out["status"].abs().sum().item()) == 0
    energies_timed = B * args.steps
    value = energies_timed / dt
    note(f"timed {args.steps} steps ({energies_timed} energies): {value:.2f} energies/s")

    # launch timing of one step (events around every launch on the solver's stream)
    ctx.profile(True)
    pkg.solve(ctx, tree, batch_of(0), want=want, out=out, sync=True, **kw)
    prof = ctx.profile_read()
    prof_bytes = ctx.profile_bytes()
    launches = ctx.profile_launches()
    ctx.profile(False)
    roof = roofline_of(prof, args.precision, prof_bytes, args.slices)
    by_phase = {}
    for kind, fl, ms, ph in launches:
        key = f"{ctx.PROFILE_PHASES[int(ph)]}/{ctx.PROFILE_KINDS[int(kind)]}"
        agg = by_phase.setdefault(key, [0, 0.0, 0.0])
        agg[0] += 1
        agg[1] += ms
        agg[2] += fl
    by_phase = {k: {"launches": v[0], "ms": round(v[1], 3),
                    "tflops": round(v[2] / (v[1] * 1e-3) / 1e12, 3) if v[2] > 0 and v[1] > 0 else None}
                for k, v in sorted(by_phase.items(), key=lambda kv: -kv[1][1])}
    total_ms = sum(v["ms"] for v in prof.values())
    note(f"dominant kernel: {roof['achieved']:.2f} TFLOP/s algorithmic = {roof['frac']:.3f} of FP64 peak")

    acc = None
    if gold and not args.no_golden:
        # the stored energies, padded to one batch so the same plan serves them
        idx = list(gold["energy_index"])
        pad = idx + [idx[-1]] * (B - len(idx) % B if len(idx) % B else 0)
        og = pkg.solve(ctx, tree, E[pad], want=want, **kw)
        n8 = len(idx)
        acc = golden_errors(np, gold, og["gr"][:n8].cpu().numpy(), og["gl"][:n8].cpu().numpy(),
                            og["trans"][:n8].cpu().numpy())
        acc["status_ok"] = int(og["status"].abs().sum().item()) == 0
        note(f"error vs stored oracle values: max {acc['max']:.2e}")
        del og

    mfma = None
    if args.alt:
        mfma = {}
        kw0 = dict(kw, precision=0)
        for name, tr in (("transverse_leaf4", pkg.Tree.from_device(dev, leaf_side=4, transverse=True)),
                         ("this_tree", tree)):
            o0 = pkg.solve(ctx, tr, batch_of(0), want=want, **kw0)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            for k in range(4):
                pkg.solve(ctx, tr, batch_of(k), want=want, out=o0, sync=False, **kw0)
            torch.cuda.synchronize()
            rate = 4 * B / (time.perf_counter() - t3)
            ctx.profile(True)
            pkg.solve(ctx, tr, batch_of(0), want=want, out=o0, sync=True, **kw0)
            p0 = ctx.profile_read()
            ctx.profile(False)
            g0 = p0["gemm"]
            a0 = g0["flops"] / (g0["ms"] * 1e-3) / 1e12
            mfma[name] = {"energies_per_s": rate, "flops_per_energy": tr.stats()["flops_per_energy"],
                          "k_zgemm_tflops": a0, "k_zgemm_frac_of_fp64_mfma_peak": a0 / FP64_MFMA_PEAK_TFLOPS,
                          "k_zgemm_avg_launch_ms": g0["ms"] / g0["launches"],
                          "k_zgemm_share_of_kernel_time": g0["ms"] / sum(v["ms"] for v in p0.values())}
            note(f"complex128 on the matrix cores, {name}: {rate:.2f} energies/s, k_zgemm {a0:.1f} TFLOP/s")
            del o0

    dense = None
    if args.dense_steps > 0:
        dense = dense_leg(pkg, np, torch, ctx, dev, E, batch_of, want, kw, args, st)

    plain = None
    if not args.no_plain:
        sub = E[: max(1, args.plain_energies)]
        kw1 = dict(kw, batch=1)
        pkg.solve(ctx, tree, sub[:1], want=want, **kw1)        # plan for one slot
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pkg.solve(ctx, tree, sub, want=want, **kw1)
        torch.cuda.synchronize()
        plain = len(sub) / (time.perf_counter() - t1)
        note(f"plain (one energy per launch sequence): {plain:.2f} energies/s")

    cpu = None
    if not args.no_cpu:
        import oracle
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        cpu_e = [0.3, -2.4]
        t2 = time.perf_counter()
        oracle.rgf.solve(dev, cpu_e, 1e-8, 0.025, 0.1, -0.1)
        cdt = time.perf_counter() - t2
        note(f"CPU oracle, {threads} threads: {len(cpu_e) / cdt:.3f} energies/s")
        single = None
        if args.cpu_single > 0:
            e1 = cpu_e[: args.cpu_single]
            with threadpool_limits(limits=1):
                t4 = time.perf_counter()
                oracle.rgf.solve(dev, e1, 1e-8, 0.025, 0.1, -0.1)
                sdt = time.perf_counter() - t4
            single = {"value": len(e1) / sdt, "unit": "energies/s", "cores": 1,
                      "sample": f"{len(e1)} energy (E={e1}), {sdt:.1f} s"}
            note(f"CPU oracle, 1 thread: {len(e1) / sdt:.4f} energies/s")
        cpu = {"value": len(cpu_e) / cdt, "unit": "energies/s", "cores": threads, "kind": "oracle",
               "sample": f"slab RGF (oracle/rgf.py), two energies (E=0.3 in the lead band, E=-2.4 outside) "
                         f"of the same {N}^3 cube, {cdt:.1f} s",
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "single_thread": single}

    prec_name = {0: "complex128", 1: "double-double fold, complex128 extraction",
                 2: "double-double fold and extraction",
                 3: f"double-double fold and extraction, products of depth >= 32 from 8-bit slices "
                    f"({args.slices or OZ_DEFAULT_SLICES} per operand) on the integer matrix cores"}[args.precision]
    line = {
        "metric": "energies/s (diag G^r,G^<), 32^3 cube, batched vs plain; % FP64 MFMA peak",
        "value": value,
        "unit": "energies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if args.precision == 0 else "c128 in/out, complex double-double inside",
        "data": "synthetic",
        "config": {"workload": f"cube{N}^3, energy grid of {NE} points in [-6,6] walked {B} at a time "
                               f"(diag G^r, diag G^<, T)",
                   "sites": int(dev.n), "grid_energies": NE, "energies_per_step": B,
                   "energies_timed": energies_timed, "leaf_side": args.leaf, "clusters": st["n_clusters"],
                   "tree": "transverse nested dissection" if args.transverse else
                           "3D nested dissection, planar separators",
                   "plain_energies_per_s": plain,
                   "batched_over_plain": value / plain if plain else None,
                   "precision": prec_name,
                   "complex_products": "3 real products (Gauss)" if args.complex3m else "4 real products",
                   "gemm_tiles": "autotuned per launch" if args.tune else "default",
                   "flops_per_energy": st["flops_per_energy"],
                   "whole_solve_tflops": value * st["flops_per_energy"] / 1e12,
                   "status_ok": ok,
                   "accuracy_vs_oracle": acc,
                   "complex128_matrix_core_path": mfma,
                   "kernel_ms_one_step": {k: round(v["ms"], 3) for k, v in prof.items() if v["ms"] > 0},
                   "kernel_ms_total_one_step": round(total_ms, 3),
                   "kernel_ms_one_step_by_phase": by_phase,
                   "dense_contacts": dense},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def write_device(np, dev, energies, path):
    """Device file of the native driver (layout documented in csrc/hsc_run.cpp)."""
    with open(path, "wb") as f:
        f.write(b"HSCDEV1\0")
        np.array([dev.n, len(dev.indices)], np.int64).tofile(f)
        np.asarray(dev.indptr, np.int64).tofile(f)
        np.asarray(dev.indices, np.int32).tofile(f)
        np.ascontiguousarray(np.asarray(dev.values, np.complex128)).view(np.float64).tofile(f)
        np.ascontiguousarray(dev.coords, np.int32).tofile(f)
        for c in dev.contacts:
            np.array([len(c.sites)], np.int64).tofile(f)
            np.asarray(c.sites, np.int64).tofile(f)
            np.array([c.lead_onsite, c.lead_hopping, c.coupling], np.float64).tofile(f)
        np.array([len(energies)], np.int64).tofile(f)
        np.asarray(energies, np.float64).tofile(f)
    note(f"device file {path}: {dev.n} sites, {len(energies)} energies")


def dense_leg(pkg, np, torch, ctx, dev, E, batch_of, want, kw, args, st):
    """The same cube and energy walk with whole-face contacts: each x face couples to a semi-infinite
    lead continuing the face lattice, so the contact self-energy is a dense face block."""
    tree = pkg.Tree.from_device(dev, leaf_side=args.leaf, dense=True)
    sd = tree.stats()
    t_setup = time.perf_counter()
    out = pkg.solve(ctx, tree, batch_of(0), want=want, **kw)
    note(f"dense contacts: set-up {time.perf_counter() - t_setup:.1f} s")
    pkg.solve(ctx, tree, batch_of(1), want=want, out=out, sync=True, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.dense_steps):
        pkg.solve(ctx, tree, batch_of(k), want=want, out=out, sync=False, **kw)
    ctx.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rate = args.batch * args.dense_steps / dt
    ok = int(out["status"].abs().sum().item()) == 0
    ctx.profile(True)
    pkg.solve(ctx, tree, batch_of(0), want=want, out=out, sync=True, **kw)
    prof = ctx.profile_read()
    ctx.profile(False)
    note(f"dense contacts: {rate:.2f} energies/s ({args.dense_steps} steps)")
    acc = None
    gpath = os.path.join(ROOT, "tests", "golden", "dense32_rgf.json")
    if dev.n == 32 ** 3 and os.path.exists(gpath) and not args.no_golden:
        gold = json.load(open(gpath))
        grid = E.cpu().numpy()
        idx = list(gold["energy_index"])
        pad = idx + [idx[-1]] * (args.batch - len(idx) % args.batch if len(idx) % args.batch else 0)
        og = pkg.solve(ctx, tree, E[pad], want=want, **kw)
        n4 = len(idx)
        acc = golden_errors(np, gold, og["gr"][:n4].cpu().numpy(), og["gl"][:n4].cpu().numpy(),
                            og["trans"][:n4].cpu().numpy())
        acc["status_ok"] = int(og["status"].abs().sum().item()) == 0
        acc["oracle"] = "slab recursion with the dense face blocks (oracle/rgf.py), energies " + \
                        ", ".join(f"{grid[i]:.4f}" for i in idx)
        note(f"dense contacts: error vs stored oracle values: max {acc['max']:.2e}")
        del og
    return {"energies_per_s": rate, "energies_timed": args.batch * args.dense_steps, "status_ok": ok,
            "flops_per_energy": sd["flops_per_energy"],
            "flops_over_per_site_leads": sd["flops_per_energy"] / st["flops_per_energy"],
            "whole_solve_tflops": rate * sd["flops_per_energy"] / 1e12,
            "max_front": sd["max_front"], "clusters": sd["n_clusters"],
            "kernel_ms_one_step": {k: round(v["ms"], 3) for k, v in prof.items() if v["ms"] > 0},
            "accuracy_vs_oracle": acc}


def dense_study(pkg, synth, np, torch, args):
    """Time per energy with whole-face (dense) and per-site (diagonal) contact self-energies, the
    cuboid experiments of Section 3.1.2: cubes N^3 (N = 16 .. 36) and elongated devices with fixed
    16 x 16 faces and growing length (Nx = 16 .. 128), at --precision, batches of --batch energies."""
    kw = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, precision=args.precision, slices=args.slices,
              complex3m=args.complex3m,
              tune=0, batch=args.batch)
    want = pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS
    E = torch.tensor(np.linspace(-1.9, 1.9, args.batch), dtype=torch.float64, device="cuda:0")
    rows = []
    shapes = [(n, n, n) for n in (16, 24, 32, 36)] + [(nx, 16, 16) for nx in (16, 32, 64, 128)]
    for shape in shapes:
        dev = synth.cuboid(*shape, onsite=np.random.default_rng(0).uniform(-0.5, 0.5, shape[0] * shape[1] * shape[2]))
        row = {"shape": list(shape), "sites": dev.n}
        for name, dense in (("per_site", False), ("dense", True)):
            ctx = pkg.Context(0)     # a context of its own: its plans (device memory) go with it
            tree = pkg.Tree.from_device(dev, leaf_side=args.leaf, dense=dense)
            out = pkg.solve(ctx, tree, E, want=want, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 2
            for _ in range(reps):
                pkg.solve(ctx, tree, E, want=want, out=out, sync=False, **kw)
            ctx.sync()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / (reps * args.batch)
            row[name] = {"ms_per_energy": dt * 1e3, "flops_per_energy": tree.stats()["flops_per_energy"],
                         "tflops": tree.stats()["flops_per_energy"] / dt / 1e12,
                         "status_ok": int(out["status"].abs().sum().item()) == 0}
            del out, tree
            ctx.close()
        note(f"{shape}: per-site {row['per_site']['ms_per_energy']:.2f} ms, dense {row['dense']['ms_per_energy']:.2f} ms "
             "per energy")
        rows.append(row)
    print(json.dumps({"metric": "ms per energy, whole-face vs per-site contacts", "value": rows[3]["dense"]["ms_per_energy"],
                      "unit": "ms per energy (36^3, dense)", "higher_is_better": False, "n_gpus": 1,
                      "dtype": "c128 in/out, complex double-double inside", "data": "synthetic",
                      "config": {"energies_per_batch": args.batch, "precision": args.precision, "leaf_side": args.leaf},
                      "rows": rows}), flush=True)


def streams_study(pkg, synth, np, torch, args):
    """Concurrent batches (hsc_solve_opts.streams) on the benchmark cube: 64 energies of the 256-point
    grid per configuration, each timed after one untimed pass that builds its plans."""
    N = args.n_side
    dev = synth.config1_device(n_side=N)
    ctx = pkg.Context(0)
    tree = pkg.Tree.from_device(dev, leaf_side=args.leaf)
    E = torch.tensor(np.linspace(-6.0, 6.0, 256)[::4].copy(), dtype=torch.float64, device="cuda:0")
    want = pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS
    kw = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, want=want, precision=args.precision, slices=args.slices,
              complex3m=args.complex3m, tune=args.tune)
    rows = []
    for batch, streams in ((16, 1), (8, 2), (4, 4)):
        out = pkg.solve(ctx, tree, E, batch=batch, streams=streams, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = pkg.solve(ctx, tree, E, batch=batch, streams=streams, out=out, **kw)
        torch.cuda.synchronize()
        rate = E.numel() / (time.perf_counter() - t0)
        ok = int(out["status"].abs().max()) == 0
        note(f"batch {batch} on {streams} stream(s): {rate:.2f} energies/s, status ok {ok}")
        rows.append({"batch": batch, "streams": streams, "energies_per_s": rate, "status_ok": ok})
    print(json.dumps({"metric": "energies/s with concurrent batches", "unit": "energies/s", "n_gpus": 1,
                      "data": "synthetic", "config": {"workload": f"cube{N}^3, 64 energies of the 256-point grid",
                                                      "precision": args.precision, "leaf_side": args.leaf},
                      "rows": rows}), flush=True)
    ctx.close()


def scf_study(pkg, synth, np, torch, args):
    """Self-consistent NEGF-Poisson loop on the benchmark cube: 64 energies in [-6, 0.5] (trapezoid
    weights), lead planes at +-0.05, coupling 0.05, mixing 0.5, 4 iterations at --precision; reports
    seconds per iteration and the share of the Poisson solve (timed on its own); then the iterations
    linear and Anderson mixing (history 4) take to a residual of 1e-8 (at most 30)."""
    N = args.n_side
    dev = synth.config1_device(n_side=N)
    ctx = pkg.Context(0)
    tree = pkg.Tree.from_device(dev, leaf_side=args.leaf)
    E = np.linspace(-6.0, 0.5, 64)
    w = np.full(64, E[1] - E[0])
    w[0] = w[-1] = 0.5 * w[0]
    kw = dict(eta=1e-8, kT=0.025, mu_L=0.05, mu_R=-0.05, precision=args.precision, slices=args.slices,
              complex3m=args.complex3m, tune=args.tune, batch=args.batch)
    pkg.scf(ctx, tree, (N, N, N), E, w, u_left=0.05, u_right=-0.05, coupling=0.05, mixing=0.5, max_iter=1, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, dens, res = pkg.scf(ctx, tree, (N, N, N), E, w, u_left=0.05, u_right=-0.05, coupling=0.05, mixing=0.5,
                           max_iter=4, **kw)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / len(res)
    rho = torch.randn(dev.n, dtype=torch.float64, device="cuda:0")
    pkg.poisson_solve(ctx, (N, N, N), rho, 0.05, -0.05)
    t1 = time.perf_counter()
    for _ in range(10):
        pkg.poisson_solve(ctx, (N, N, N), rho, 0.05, -0.05)
    tp = (time.perf_counter() - t1) / 10
    note(f"self-consistent loop on the {N}^3 cube: {dt:.3f} s per iteration (64 energies), Poisson solve "
         f"{tp * 1e3:.3f} ms ({tp / dt:.2e} of an iteration), residuals {np.array2string(res, precision=3)}")
    to_tol = {}
    u_tol = {}
    for name, hist in (() if args.scf_quick else (("linear", 0), ("anderson4", 4))):
        ut, _, rt = pkg.scf(ctx, tree, (N, N, N), E, w, u_left=0.05, u_right=-0.05, coupling=0.05, mixing=0.5,
                            max_iter=30, tol=1e-8, history=hist, **kw)
        to_tol[name] = {"iterations": len(rt), "last_residual": float(rt[-1])}
        u_tol[name] = ut
        note(f"{name} mixing: {len(rt)} iterations to residual {rt[-1]:.2e}")
    u_diff = None if args.scf_quick else float((u_tol["linear"] - u_tol["anderson4"]).abs().max())
    print(json.dumps({"metric": "seconds per self-consistent iteration", "value": dt, "unit": "s",
                      "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                      "dtype": "c128 in/out, complex double-double inside",
                      "config": {"workload": f"cube{N}^3, 64 energies in [-6, 0.5], 4 iterations",
                                 "precision": args.precision, "leaf_side": args.leaf},
                      "poisson_ms": tp * 1e3, "residuals": res.tolist(), "to_1e-8": to_tol,
                      "u_linear_vs_anderson": u_diff,
                      "u_range": [float(u.min()), float(u.max())], "density_mean": float(dens.mean())}),
          flush=True)
    ctx.close()


def orbital_study(pkg, synth, np, torch, args):
    """Multi-orbital site blocks (10 orbitals per site, random blocks: the block structure of the
    paper's sp3d5s* nanowires): wires of 4 x 4 and 6 x 6 sites across and 32 .. 128 sites long, per-site
    leads on every orbital of the end faces, at --precision, batches of --batch energies in [-4, 4]."""
    kw = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, precision=args.precision, slices=args.slices,
              complex3m=args.complex3m,
              tune=0, batch=args.batch)
    want = pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS
    E = torch.tensor(np.linspace(-4.0, 4.0, args.batch), dtype=torch.float64, device="cuda:0")
    rows = []
    for cross in (4, 6):
        for length in (32, 64, 128):
            dev = synth.orbital_cuboid(length, cross, cross, 10, seed=length + cross)
            ctx = pkg.Context(0)
            tree = pkg.Tree.from_device(dev, leaf_side=2)
            st = tree.stats()
            out = pkg.solve(ctx, tree, E, want=want, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                pkg.solve(ctx, tree, E, want=want, out=out, sync=False, **kw)
            ctx.sync()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / (2 * args.batch)
            rows.append({"sites": [length, cross, cross], "orbitals": 10, "unknowns": dev.n,
                         "ms_per_energy": dt * 1e3, "flops_per_energy": st["flops_per_energy"],
                         "tflops": st["flops_per_energy"] / dt / 1e12, "max_cluster": st["max_cluster"],
                         "status_ok": int(out["status"].abs().sum().item()) == 0})
            note(f"10-orbital wire {length} x {cross} x {cross} ({dev.n} unknowns): {dt * 1e3:.2f} ms per energy, "
                 f"{rows[-1]['tflops']:.2f} TFLOP/s")
            del out, tree
            ctx.close()
    print(json.dumps({"metric": "ms per energy, 10-orbital wires", "value": rows[-1]["ms_per_energy"],
                      "unit": "ms per energy (128 x 6 x 6 sites x 10 orbitals)", "higher_is_better": False,
                      "n_gpus": 1, "dtype": "c128 in/out, complex double-double inside", "data": "synthetic",
                      "config": {"energies_per_batch": args.batch, "precision": args.precision}, "rows": rows}),
          flush=True)


def trilayer_study(pkg, synth, np, torch, args):
    """Graphene / BN / graphene trilayer (116 x 115 x 3 sites, in-plane nested dissection, leaves <= 8
    across), 512 energies in [-3, 3] eV, unguarded, at --precision; error against the stored RGF values
    at 6 energies."""
    dev = synth.trilayer()
    tree = pkg.Tree.from_device(dev, leaf_side=8)
    ctx = pkg.Context(0)
    E = torch.tensor(np.linspace(-3.0, 3.0, 512), dtype=torch.float64, device="cuda:0")
    kw = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, precision=args.precision, slices=args.slices,
              complex3m=args.complex3m,
              tune=args.tune, want=pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS)
    out = pkg.solve(ctx, tree, E, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pkg.solve(ctx, tree, E, out=out, sync=False, **kw)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "trilayer_rgf.json")))
    sites = np.array(gold["sites"])
    ref = np.array(gold["gr_re"]) + 1j * np.array(gold["gr_im"])
    gr = out["gr"].cpu().numpy()
    errs = [float(np.abs(gr[i][sites] - ref[k]).max() / np.abs(ref[k]).max())
            for k, i in enumerate(gold["energy_index"])]
    note(f"trilayer: {512 / dt:.1f} energies/s, max error {max(errs):.1e}")
    print(json.dumps({"metric": "energies/s (diag G^r, G^<, T), trilayer 40,020 sites", "value": 512 / dt,
                      "unit": "energies/s", "higher_is_better": True, "n_gpus": 1,
                      "dtype": "c128" if args.precision == 0 else "c128 in/out, complex double-double inside",
                      "data": "synthetic",
                      "config": {"workload": "graphene/BN/graphene 116x115x3 x 512 energies in [-3, 3] eV, unguarded",
                                 "precision": args.precision,
                                 "flops_per_energy": tree.stats()["flops_per_energy"],
                                 "gr_rel_err_at_stored_energies": errs}}),
          flush=True)


def guard_study(pkg, synth, np, torch, args):
    """32^3 cube, 256 energies in [-6, 6], complex128 on the matrix cores (precision 0) on the 3D tree
    (leaf 8) with the growth guard (tau 100, up to 8 rounds of merges), in chunks of 32 energies with
    a progress line each; error at the stored oracle energies."""
    dev = synth.config1_device()
    tree = pkg.Tree.from_device(dev, leaf_side=8)
    ctx = pkg.Context(0)
    grid = np.linspace(-6.0, 6.0, 256)
    E = torch.tensor(grid, dtype=torch.float64, device="cuda:0")
    kw = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, precision=0, complex3m=args.complex3m, tune=0,
              want=pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS, guard=True, guard_tau=100.0, guard_rounds=8)
    t0 = time.perf_counter()
    gr, gl, tr, stv = [], [], [], []
    for c in range(0, 256, 32):
        o = pkg.solve(ctx, tree, E[c:c + 32], **kw)
        gr.append(o["gr"].cpu().numpy()); gl.append(o["gl"].cpu().numpy()); tr.append(o["trans"].cpu().numpy())
        stv.append(o["status"].cpu().numpy())
        note(f"guarded energies {c}..{c + 31} done, {time.perf_counter() - t0:.1f} s, "
             f"unstable {int((stv[-1] == -7).sum())}")
    dt = time.perf_counter() - t0
    gr, gl, tr, stv = (np.concatenate(x) for x in (gr, gl, tr, stv))
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "cube32_sampled.json")))
    idx = gold["energy_index"]
    acc = golden_errors(np, gold, gr[idx], gl[idx], tr[idx])
    print(json.dumps({"metric": "guarded complex128 solve, 32^3 x 256 energies", "value": 256 / dt,
                      "unit": "energies/s", "higher_is_better": True, "n_gpus": 1, "dtype": "c128", "data": "synthetic",
                      "config": {"seconds": dt, "unstable": int((stv == -7).sum()), "failed": int((stv < 0).sum()),
                                 "accuracy_vs_oracle": acc}}), flush=True)


def uneven_study(pkg, synth, np, torch, args):
    """The first D of the 64 uneven cuboids (sides 16..48, on-site N(0, 0.3^2)) on transverse trees,
    the same energies (linspace(-6, 6, n)) for all: one hsc_solve_batch call (devices packed into
    forests sharing launches) against one hsc_solve per device."""
    D, NE = args.uneven, args.uneven_energies
    ctx = pkg.Context(0)
    devs = synth.config2_devices(which=range(D))
    trees = [pkg.Tree.from_device(d, leaf_side=4, transverse=True) for d in devs]
    # the grid as numpy builds it (torch.linspace differs from it by an ulp at some points)
    E = torch.tensor(np.linspace(-6.0, 6.0, NE), dtype=torch.float64, device="cuda:0")
    # no tile tuning here: with more devices than cached plans, plans are rebuilt per call
    kw = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, precision=0, complex3m=args.complex3m, tune=0,
              want=pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS)
    flops = sum(t.stats()["flops_per_energy"] for t in trees) * NE

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    outs = [pkg.solve(ctx, t, E, **kw) for t in trees]
    t_loop = timed(lambda: [pkg.solve(ctx, t, E, out=o, sync=False, **kw) for t, o in zip(trees, outs)])
    note(f"one device at a time: {D * NE / t_loop:.2f} device-energies/s")
    del outs
    bo = pkg.solve_batch(ctx, trees, E, **kw)
    t_batch = timed(lambda: pkg.solve_batch(ctx, trees, E, outs=bo, **kw))
    note(f"forest batch: {D * NE / t_batch:.2f} device-energies/s")
    ok = all(int(o["status"].abs().sum().item()) == 0 for o in bo)
    print(json.dumps({"metric": "uneven devices: device-energies/s (diag G^r, G^<, T)", "value": D * NE / t_batch,
                      "unit": "device-energies/s", "higher_is_better": True, "n_gpus": 1, "dtype": "c128",
                      "data": "synthetic",
                      "config": {"workload": f"first {D} of 64 uneven cuboids (sides 16..48) x {NE} energies",
                                 "sides": [list(map(int, s)) for s in synth.config2_sizes()[:D]],
                                 "one_device_at_a_time": D * NE / t_loop, "status_ok": ok,
                                 "whole_solve_tflops": flops / t_batch / 1e12}}), flush=True)


def config2_full(pkg, synth, np, torch, args):
    """The uneven-device workload at its size: 64 cuboids (sides 16..48, on-site N(0, 0.3^2)) x 128
    energies in [-6, 6], every device on its 3D nested-dissection tree (leaves <= 8), at --precision;
    hsc_solve_batch over four devices per call (plans built inside the timed pass)."""
    NE = 128
    ctx = pkg.Context(0)
    E = torch.tensor(np.linspace(-6.0, 6.0, NE), dtype=torch.float64, device="cuda:0")
    kw = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, precision=args.precision, slices=args.slices,
              complex3m=args.complex3m, tune=0,
              want=pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS)
    sizes = synth.config2_sizes()
    flops, ok, t0 = 0.0, True, time.perf_counter()
    for g in range(0, 64, 4):
        devs = [synth.config2_devices(which=[d])[0] for d in range(g, g + 4)]
        trees = [pkg.Tree.from_device(d, leaf_side=8) for d in devs]
        flops += sum(t.stats()["flops_per_energy"] for t in trees) * NE
        outs = pkg.solve_batch(ctx, trees, E, **kw)
        torch.cuda.synchronize()
        ok = ok and all(int(o["status"].abs().sum().item()) == 0 for o in outs)
        note(f"devices {g}..{g + 3} done ({sum(d.n for d in devs)} sites), {time.perf_counter() - t0:.1f} s")
        del outs, trees, devs
    dt = time.perf_counter() - t0
    note(f"64 devices x {NE} energies: {64 * NE / dt:.2f} device-energies/s, {flops / dt / 1e12:.2f} TFLOP/s")
    print(json.dumps({"metric": "uneven devices at full size: device-energies/s (diag G^r, G^<, T)",
                      "value": 64 * NE / dt, "unit": "device-energies/s", "higher_is_better": True, "n_gpus": 1,
                      "dtype": "c128 in/out, complex double-double inside" if args.precision else "c128",
                      "data": "synthetic",
                      "config": {"workload": "64 uneven cuboids (sides 16..48, N(0, 0.3^2)) x 128 energies in [-6, 6]",
                                 "sites_total": int(sum(int(np.prod(s)) for s in sizes)), "seconds": dt,
                                 "precision": args.precision, "tree": "3D nested dissection, leaves <= 8",
                                 "whole_solve_tflops": flops / dt / 1e12, "status_ok": ok}}), flush=True)


def learned_grid_study(pkg, synth, np):
    """Surrogate network trained on solver outputs of 40 disordered cubes (N in 24..32,
    sigma ~ U[0, 0.5], 50 energies each in [-6, 6]); charge of three N = 32, sigma = 0.3 cubes
    on 512 of 4096 candidate energies, against the dense grid (every candidate in the lead band)."""
    from paper_1702_05167_amd import learned_grid as lg
    ctx = pkg.Context(0)
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    items = []
    for d in range(40):
        N = int(rng.integers(24, 33))
        sig = float(rng.uniform(0.0, 0.5))
        dev = synth.learned_grid_device(N, sig, 1000 + d)
        items.append(dict(tree=pkg.Tree.from_device(dev, leaf_side=4, transverse=True), n_sites=dev.n, sigma=sig,
                          nx=N, ny=N))
    X, Y = lg.dataset(ctx, items, 50, seed=1)
    del items
    t_data = time.perf_counter() - t0
    note(f"training set {X.shape[0]} samples in {t_data:.1f} s")
    sur = lg.Surrogate(ctx, seed=0)
    t1 = time.perf_counter()
    hist = sur.fit(X, Y, epochs=300, batch=200)
    t_fit = time.perf_counter() - t1
    note(f"fit {len(hist)} Adam steps in {t_fit:.2f} s, loss {hist[0]:.3f} -> {hist[-1]:.4f}")
    cand = np.linspace(-6.0, 6.0, 4096)
    runs = []
    for seed in (100, 101, 102):
        dev = synth.learned_grid_device(32, 0.3, seed)
        it = dict(tree=pkg.Tree.from_device(dev, leaf_side=4, transverse=True), n_sites=dev.n, sigma=0.3, nx=32, ny=32)
        r = lg.study(ctx, sur, it, cand, 512, (-2.0, 2.0), budget=64)
        r["seed"] = seed
        # solves needed to reach the 1e-4 charge tolerance: guided (proposal + refinement), the same
        # refinement from evenly spaced points, evenly spaced in-band points, and the plain grid
        ec = lg.equal_cost(ctx, sur, it, cand, (-2.0, 2.0), (64, 96, 128, 192, 256, 384, 512, 768))
        r["equal_cost"] = ec
        plain = {}
        for K in (64, 128, 256, 512, 1024, 2048):
            g = np.arange(0, cand.size, max(cand.size // K, 1))
            e = lg.Integrator(ctx, it["tree"], it["n_sites"], cand, (-2.0, 2.0))
            q = e.charge(g)
            plain[K] = {"in_band_solves": e.cost(g), "rel_err": abs(q - r["dense"]["charge"]) / abs(r["dense"]["charge"])}
        r["plain_grid"] = plain
        ok_plain = [v["in_band_solves"] for v in plain.values() if v["rel_err"] <= 1e-4]
        r["solves_to_1e-4"] = dict(ec["solves_to_tol"], plain=min(ok_plain) if ok_plain else None)
        runs.append(r)
        note(f"device seed {seed}: guided {r['guided']['rel_err']:.2e} ({r['guided']['solves']} solves), "
             f"uniform {r['uniform']['rel_err']:.2e} ({r['uniform']['solves']}), dense {r['dense']['solves']} solves; "
             f"solves to 1e-4: {r['solves_to_1e-4']}")
    worst = max(r["guided"]["rel_err"] for r in runs)
    line = {"metric": "learned energy grid: charge error vs dense grid (32^3, sigma 0.3, 3 devices)",
            "value": worst, "unit": "relative error", "higher_is_better": False, "n_gpus": 1,
            "dtype": "f32 net / c128 solve",
            "data": "synthetic",
            "config": {"workload": "MLP 4-256-256-2 trained on 2000 solver samples (40 cubes N 24..32); 512 of 4096 "
                                   "candidates in [-6, 6]; charge over the open lead band (-2, 2)",
                       "train_seconds": t_fit, "data_seconds": t_data, "loss_first": float(hist[0]),
                       "loss_last": float(hist[-1]), "adam_steps": len(hist)},
            "runs": runs}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
