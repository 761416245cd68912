"""Benchmark of the tree-based column-density sweep on one MI355X.

A step is one pass of the whole hot path over the resident synthetic field:
rebuild the pyramid from the leaf densities (cd_tree_update), then the column
sweep with the fused screening epilogue (cd_column_densities: N_H[n_leaf][D]
and chi[n_leaf]).  The weight tables are precalculated once, outside the
timed region, as in the method (Sect. 3.3).

Default workload: the largest single-GPU configuration, a 512^3 uniform grid
(134M leaves, 10-level pyramid), log-normal turbulent field sigma_ln n = 1.5,
mean 10 cm^-3, box 10 pc, 48 HEALPix sectors (N_side = 2), FP32.  The same
resident input is also timed with the split-precision forms (bf16 / fp16 hi +
lo on the matrix cores), the in-situ reference points and 12 sectors, reported
under "forms" with their speed-up and error against an oracle sample.
--level 8 --nside 1: the 256^3 grid with 12 sectors; --workload amr: the
adaptive tree (128^3 base + 2 levels, D = 48).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def alg_bytes_step(tin, D: int) -> float:
    """Algorithmic HBM bytes of one step: read every leaf density once (4 B),
    write and read back the coarse cells of the pyramid once (4 B each: every
    level below the leaves of a uniform grid, the base levels below B and
    every refined cell of an adaptive tree), write the row of N (4 D B) and
    chi (4 B) of every leaf.  Intermediates of this implementation (external
    rows, coarse tables) are not counted."""
    if tin.base_level == tin.max_level:
        coarse = sum(8 ** l for l in range(tin.max_level))
    else:
        coarse = sum(8 ** l for l in range(tin.base_level)) + sum(p.shape[0] for p in tin.oct_parents)
    return tin.n_leaf * (4.0 + 4.0 * D + 4.0) + 4.0 * coarse


def measured_traffic(key: str):
    """HBM bytes per launch from the committed rocprofv3 counter runs
    (profiles/traffic.json), or None if the kernel source changed since."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[key]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    return rec["traffic_bytes"] if hashlib.sha256(src).hexdigest() == rec["sha256"] else None


PREC = {"fp32": 0, "bf16x2": 1, "fp16x2": 2}
MFMA_PEAK_TFLOPS = 2500.0  # dense bf16 / fp16


def hbm_ceiling(torch, n_floats):
    """Plain torch copy and fill on this GPU, sized like the row kernel's
    output (at most 2^31 floats, well past the last-level cache): the rate a
    streaming kernel reaches here, as context for roofline.frac (whose peak
    is the published 8 TB/s)."""
    n = int(min(n_floats, 1 << 31))
    a = torch.ones(n, device="cuda:0")
    b = torch.empty_like(a)
    out = {"n_bytes": n * 4}
    for name, fn, nbytes in (("copy", lambda: b.copy_(a), 8 * n), ("fill", lambda: b.fill_(1.0), 4 * n)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            fn()
        e1.record()
        e1.synchronize()
        out[f"{name}_GBps"] = nbytes / (e0.elapsed_time(e1) / 20 * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=["uniform", "amr", "sphere", "surrogate"], default="uniform")
    ap.add_argument("--sphere-sample", type=int, default=1500,
                    help="sphere: midplane leaves checked against the exact-ray reference")
    ap.add_argument("--amr-threshold", type=float, default=100.0,
                    help="adaptive tree: refine cells with averaged n above this (cm^-3)")
    ap.add_argument("--train-fields", type=int, default=16, help="surrogate: seeded 256^3 training fields")
    ap.add_argument("--train-steps", type=int, default=6000, help="surrogate: Adam steps")
    ap.add_argument("--train-batch", type=int, default=8192, help="surrogate: level-7 cells per step")
    ap.add_argument("--level", type=int, default=9, help="uniform grid of 2^level cells per axis")
    ap.add_argument("--nside", type=int, default=2, help="HEALPix Nside, D = 12 Nside^2")
    ap.add_argument("--precision", choices=list(PREC), default="fp32")
    ap.add_argument("--no-forms", action="store_true", help="skip timing the other precision forms")
    ap.add_argument("--cpu-sample-octs", type=int, default=0,
                    help="uniform grids: octs timed with the CPU oracle (bounded sample; default "
                         "2e8 / (8 D) octs, about 10-30 s of oracle work)")
    ap.add_argument("--cpu-sample-leaves", type=int, default=400000,
                    help="adaptive tree: leaves timed with the CPU oracle (bounded sample)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-reference", action="store_true",
                    help="run only an elementwise copy of known size (256 MiB read, 256 MiB written), the "
                         "reference that scales the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.copy_reference:
        import torch
        a = torch.ones(1 << 26, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference": "torch.mul(a, 2, out=b)", "bytes_read": a.numel() * 4,
                          "bytes_written": b.numel() * 4, "launches": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU sharding is a design note only",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "surrogate":
        bench_surrogate(args)
        return

    import torch

    from paper_1410_0624_amd import colden, synth

    dev = torch.device("cuda:0")
    sphere = args.workload == "sphere"
    amr = args.workload in ("amr", "sphere")
    nside = args.nside
    t0 = time.time()
    if sphere:
        tin = synth.workload_sphere()
        wl = ("uniform sphere (R 12.5 pc, 1000 cm^-3 inside, 10 cm^-3 outside, box 50 pc): 128^3 base, "
              "every cell with sphere matter refined to 512^3 effective")
        L = tin.max_level
    elif amr:
        tin = synth.workload_amr(threshold=args.amr_threshold)
        wl = (f"AMR tree: 128^3 base + 2 refined levels on cells with averaged n > {args.amr_threshold:g} cm^-3 "
              f"(log-normal, sigma_ln n=2, mean 10 cm^-3, generated at 512^3, box 20 pc, seed 3)")
        L = tin.max_level
    else:
        L = args.level
        seed = {8: 2, 9: 4}.get(L, 2)
        tin = synth.workload_uniform(L, sigma=1.5, mean=10.0, seed=seed)
        wl = (f"uniform {1 << L}^3 log-normal turbulent field (sigma_ln n=1.5, mean 10 cm^-3, "
              f"box 10 pc, seed {seed})")
    # the sphere test uses the paper's own direction sets (M x N, axes)
    dirs = (colden.directions(colden.CD_DIR_PAPER_MN, 3, 4) if sphere
            else colden.directions(colden.CD_DIR_HEALPIX, nside))
    sets = {}
    if sphere:
        sets = {"axes6": colden.directions(colden.CD_DIR_AXES6, 0), "mn3x4": dirs,
                "mn5x8": colden.directions(colden.CD_DIR_PAPER_MN, 5, 8),
                "mn7x12": colden.directions(colden.CD_DIR_PAPER_MN, 7, 12),
                "healpix2": colden.directions(colden.CD_DIR_HEALPIX, 2)}
    D = dirs.shape[0]
    print(f"# generated workload in {time.time() - t0:.1f}s: {tin.n_leaf} leaves, D={D}",
          file=sys.stderr, flush=True)

    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    N = torch.empty((tin.n_leaf, D), dtype=torch.float32, device=dev)
    chi = torch.empty(tin.n_leaf, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    # the tree's workspace (a torch tensor) holds the sweep's buffers for up to
    # max_dirs directions; its second stream is a torch stream
    tree = colden.Tree(tin, leaf, max_dirs=max([D, 12] + [u.shape[0] for u in sets.values()]))
    rng = np.random.default_rng(0)
    check = rng.choice(tin.n_leaf, size=min(2000, tin.n_leaf), replace=False)

    def measure(prec: str, mode: int = colden.CD_PRECALC73, u=None, Nout=None, packed: bool = False) -> dict:
        u = dirs if u is None else u
        Nout = N if Nout is None else Nout
        w = colden.Weights(u, precision=PREC[prec], mode=mode)
        if packed:  # the columns as 16-bit log codes (half the output bytes)
            Nout = torch.empty((tin.n_leaf, u.shape[0]), dtype=torch.int16, device=dev)

        def step():
            tree.update(leaf)
            if packed:
                colden.column_densities_log16(tree, w, Nout, chi)
            else:
                colden.column_densities(tree, w, Nout, chi)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        # timed region: K whole steps
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            step()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_step = ev0.elapsed_time(ev1) / args.steps
        # stage durations from the library's HIP events (recorded on the
        # stream each stage runs on), averaged over as many steps
        tree.profile(True)
        stages = {k: [] for k in colden.STAGES}
        for _ in range(args.steps):
            step()
            for k, v in tree.stage_ms().items():
                stages[k].append(v)
        tree.profile(False)
        torch.cuda.synchronize()
        out = {"ms_per_step": ms_step, "value": tin.n_leaf * u.shape[0] / (ms_step * 1e-3),
               "stages_ms": {k: float(np.mean(v)) for k, v in stages.items()},
               "sample": (colden.decode_log16(Nout[torch.from_numpy(check).to(dev)]) if packed else
                          Nout[torch.from_numpy(check).to(dev)]).cpu().numpy().astype(np.float64),
               "split_steps": w.split_steps()}
        w.close()
        if packed:
            del Nout
            torch.cuda.empty_cache()
        return out

    main_form = measure(args.precision)
    forms = {args.precision: main_form}
    insitu = None
    if not args.no_forms and args.precision == "fp32":
        # in-situ reference points (every shell seen from the oct centre):
        # timed on the same field, and compared with the precalculated form
        # over every output
        N_prec, chi_prec = N.clone(), chi.clone()
        insitu = measure("fp32", mode=colden.CD_INSITU)
        dchi = (chi_prec - chi).abs()
        flatN, flatP = N.reshape(-1), N_prec.reshape(-1)
        tot, cnt = 0.0, 0
        for k in range(0, flatN.numel(), 1 << 28):
            a, b = flatN[k:k + (1 << 28)].double(), flatP[k:k + (1 << 28)].double()
            tot += float(((b - a).abs() / a).sum())
            cnt += a.numel()
        g = torch.Generator(device=dev)
        g.manual_seed(0)
        pick = torch.randint(0, flatN.numel(), (1 << 20,), device=dev, generator=g)
        dn = ((flatP[pick].double() - flatN[pick].double()).abs() / flatN[pick].double()).cpu().numpy()
        insitu["vs_precalc"] = {"mean_abs_dchi": float(dchi.double().mean()), "max_abs_dchi": float(dchi.max()),
                                "mean_rel_dN": tot / cnt, "p99_rel_dN_sample": float(np.percentile(dn, 99)),
                                "what": "|chi_prec - chi_insitu| over every leaf; |N_prec - N_insitu| / N_insitu "
                                        "over every output (p99 on 2^20 sampled outputs)"}
        del N_prec, chi_prec
        # the Sect. 4.4 comparison's own directions: theta_1 = arccos(1 - 1/M)
        # at phi = 0 for M = 3, 5, 7, precalculated against in situ over
        # every leaf of the field
        d3 = np.array([[np.sqrt(1 - (1 - 1 / M) ** 2), 0.0, 1 - 1 / M] for M in (3, 5, 7)])
        N3 = {}
        for mode in (colden.CD_PRECALC73, colden.CD_INSITU):
            w3 = colden.Weights(d3, mode=mode)
            N3[mode] = torch.empty((tin.n_leaf, 3), dtype=torch.float32, device=dev)
            colden.column_densities(tree, w3, N3[mode])
            w3.close()
        rel3 = ((N3[colden.CD_PRECALC73].double() - N3[colden.CD_INSITU].double()).abs()
                / N3[colden.CD_INSITU].double())
        insitu["vs_precalc"]["theta1_phi0"] = {
            f"M={M}": {"mean_rel_dN": float(rel3[:, i].mean()),
                       "p99_rel_dN": float(torch.quantile(rel3[::max(1, tin.n_leaf // (1 << 22)), i].float(), 0.99)),
                       "max_rel_dN": float(rel3[:, i].max())} for i, M in enumerate((3, 5, 7))}
        del N3, rel3
        print(f"# in-situ form: {insitu['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    if not args.no_forms:
        for p in PREC:
            if p == args.precision or (amr and p == "fp16x2" and D not in (6, 12, 24, 40, 48)):
                continue
            forms[p] = measure(p)
            print(f"# form {p}: {forms[p]['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    if not args.no_forms and not amr and D % 4 == 0 and L >= 5:
        # opt-in output format: 16-bit log codes of N (|d ln N| <= 3.4e-4 by
        # construction), FP32 and split sums
        for p in ("fp32", "bf16x2"):
            forms[f"{p}_log16"] = measure(p, packed=True)
            print(f"# form {p}_log16: {forms[f'{p}_log16']['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    d12 = None
    if not args.no_forms and not amr and D != 12:
        # the same field with 12 sectors (HEALPix N_side = 1)
        dirs12 = colden.directions(colden.CD_DIR_HEALPIX, 1)
        N12 = torch.empty((tin.n_leaf, 12), dtype=torch.float32, device=dev)
        d12 = measure(args.precision, u=dirs12, Nout=N12)
        del N12
        torch.cuda.empty_cache()
        print(f"# 12 sectors: {d12['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    stage_ms = main_form["stages_ms"]
    ms_step = main_form["ms_per_step"]
    value = main_form["value"]

    # the dominant kernel is the one writing the rows of N and chi; its
    # numerator is the algorithmic bytes of the whole step (leaf, pyramid, N,
    # chi), its time the sum of its launches (one per z-slab)
    if amr:
        kname = (f"k_target_leaves<{D}> (a lane per target: external row + coarse table, internal+local, N and chi rows)"
                 if D in (6, 12, 24, 40, 48) else
                 "k_target_octs (per target oct, a lane per direction: external row + coarse table, internal+local, "
                 "N and chi rows)")
    else:
        kname = (f"k_target_rows_mfma<{D}> (internal+local on the matrix cores, N and chi rows)" if D in (24, 40, 48)
                 else f"k_target_rows<{D}> (internal+local, N and chi rows)")
    step_bytes = alg_bytes_step(tin, D)
    achieved = step_bytes / (stage_ms["rows"] * 1e-3) / 1e9

    cpu = None
    ref_check = None
    ref_check_insitu = None
    ref_check12 = None
    e1 = None
    if not args.no_cpu:
        import oracle
        tr = oracle.Tree(tin)
        threads = os.cpu_count() or 1
        if amr:
            tg = rng.choice(tin.n_leaf, size=min(args.cpu_sample_leaves, tin.n_leaf), replace=False)
            what = f"{tg.shape[0]} random leaves of the same tree"
        else:
            n1 = 1 << (L - 1)
            n_sample = args.cpu_sample_octs or int(2e8 / (8 * D))
            octs = rng.choice(n1 ** 3, size=min(n_sample, n1 ** 3), replace=False)
            ax, ay, az = octs % n1, (octs // n1) % n1, octs // (n1 * n1)
            n = 1 << L
            tg = np.concatenate([((2 * az + (o >> 2)) * n + 2 * ay + ((o >> 1) & 1)) * n + 2 * ax + (o & 1)
                                 for o in range(8)]).astype(np.int64)
            what = f"{octs.shape[0]} random octs ({tg.shape[0]} leaves) of the same field"
        t0 = time.time()
        ref = tr.columns(dirs, tg, nthreads=threads)
        oracle.screening(ref)
        dt = time.time() - t0
        cpu = {"value": float(tg.shape[0] * D / dt), "unit": "cell*dir/s", "cores": threads,
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{what}, FP64 OpenMP oracle, {dt:.1f} s"}
        # the same oracle on one thread, over 1/32 of the sample (whole octs
        # on uniform grids)
        tg1 = (tg[: max(tg.shape[0] // 32, 8)] if amr else
               tg.reshape(8, -1)[:, : max(tg.shape[0] // 256, 1)].ravel())
        t0 = time.time()
        oracle.screening(tr.columns(dirs, tg1, nthreads=1))
        dt1 = time.time() - t0
        cpu["one_thread"] = {"value": float(tg1.shape[0] * D / dt1), "unit": "cell*dir/s", "cores": 1,
                             "sample": f"{tg1.shape[0]} of those leaves, {dt1:.1f} s"}
        ref_check = tr.columns(dirs, check, nthreads=threads)
        ref_check_insitu = tr.columns(dirs, check, mode=oracle.INSITU, nthreads=threads) if insitu else None
        ref_check12 = tr.columns(colden.directions(colden.CD_DIR_HEALPIX, 1), check, nthreads=threads) if d12 else None
        if sphere:
            # the paper's first test: midplane chi of the method against
            # exact rays (768 HEALPix N_side = 8 centres per target through
            # every leaf), for its four direction sets
            mid = synth.midplane_leaves(tin)
            ms = np.sort(np.random.default_rng(11).choice(mid, size=min(args.sphere_sample, mid.size),
                                                          replace=False))
            t1 = time.time()
            chi_ref = oracle.screening(tr.raymarch(oracle.dirs_healpix(8), ms, nthreads=threads))
            t_ray = time.time() - t1
            e1 = {"targets": f"{ms.size} random leaves just below the z = box/2 plane",
                  "reference": "exact rays: 768 HEALPix N_side = 8 centres per target, FP64 oracle",
                  "raymarch_s": t_ray, "sets": {}}
            paper = {"axes6": 0.036, "mn3x4": 0.017, "mn5x8": 0.014, "mn7x12": 0.018}
            for name, u in sets.items():
                w = colden.Weights(u)
                Ns = torch.empty((tin.n_leaf, u.shape[0]), dtype=torch.float32, device=dev)
                cs = torch.empty(tin.n_leaf, dtype=torch.float32, device=dev)
                colden.column_densities(tree, w, Ns, cs)
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ev0.record(stream)
                for _ in range(3):
                    colden.column_densities(tree, w, Ns, cs)
                ev1.record(stream)
                torch.cuda.synchronize()
                ms_sweep = ev0.elapsed_time(ev1) / 3
                got = cs[torch.from_numpy(ms).to(dev)].cpu().numpy().astype(np.float64)
                ref_tree = tr.columns(u, ms[:300], nthreads=threads)
                gotN = Ns[torch.from_numpy(ms[:300]).to(dev)].cpu().numpy().astype(np.float64)
                d = np.abs(got - chi_ref)
                e1["sets"][name] = {"D": int(u.shape[0]), "sweep_ms": ms_sweep,
                                    "cell_dir_per_s": tin.n_leaf * u.shape[0] / (ms_sweep * 1e-3),
                                    "mean_abs_dchi_vs_rays": float(d.mean()), "max_abs_dchi_vs_rays": float(d.max()),
                                    "paper_mean_abs_dchi": paper.get(name),
                                    "max_rel_err_vs_oracle_tree": float(np.max(np.abs(gotN - ref_tree) / ref_tree))}
                w.close()
                del Ns, cs

    def errs(f):
        if ref_check is None:
            return None, None
        got = f["sample"]
        return (float(np.max(np.abs(got - ref_check) / ref_check)),
                float(np.max(np.abs(np.log(got) - np.log(ref_check)))))

    n_tiles = ((1 << (L - 1)) // 16) ** 3 if not amr else 0
    forms_out = {}
    for p, f in forms.items():
        rel, lnerr = errs(f)
        o = {"ms_per_step": f["ms_per_step"], "value": f["value"],
             "speedup_vs_fp32": (forms["fp32"]["ms_per_step"] / f["ms_per_step"]) if "fp32" in forms else None,
             "external_ms": f["stages_ms"]["external"], "sweep_ms": f["stages_ms"]["sweep"],
             "max_rel_err_vs_oracle": rel, "max_abs_dlnN_vs_oracle": lnerr,
             "oracle_sample": f"{check.shape[0]} random leaves"}
        if p.endswith("_log16"):
            o["output_format"] = ("16-bit log codes, N = 2^(40 + c/1024): 2 B per output instead of 4 "
                                  "(an output-format change; the sums and chi are those of the unpacked form)")
        if p not in ("fp32", "fp32_log16") and not amr and f["stages_ms"]["external"] > 0:
            flops = f["split_steps"] * 4 * 3 * (16 * 16 * 32 * 2) * n_tiles
            tf = flops / (f["stages_ms"]["external"] * 1e-3) / 1e12
            o["mfma"] = {"kernel": f"k_external_mfma<{p.split('_')[0]}>", "flops_per_launch": flops, "achieved_tflops": tf,
                         "peak_tflops": MFMA_PEAK_TFLOPS, "frac": tf / MFMA_PEAK_TFLOPS}
        forms_out[p] = o
    if insitu is not None:
        o = {"ms_per_step": insitu["ms_per_step"], "value": insitu["value"],
             "slowdown_vs_precalc": insitu["ms_per_step"] / main_form["ms_per_step"],
             "external_ms": insitu["stages_ms"]["external"], "insitu_coarse_ms": insitu["stages_ms"]["coarse"],
             "rows_ms": insitu["stages_ms"]["rows"], "vs_precalc": insitu["vs_precalc"],
             # the paper's timing table (Sect. 4.4): whole RAMSES runs with
             # screening over runs without, in situ / precalculated, on CPUs
             "paper_context": {"t_sim_over_t0_insitu_precalc": {"12": [7.9, 1.6], "40": [15.8, 2.4],
                                                                 "84": [26.3, 3.3]},
                               "what": "context only: whole-simulation time ratios of the paper's CPU runs; "
                                       "slowdown_vs_precalc here is the column sweep alone on one GPU"}}
        if ref_check_insitu is not None:
            o["max_rel_err_vs_oracle_insitu"] = float(np.max(np.abs(insitu["sample"] - ref_check_insitu)
                                                             / ref_check_insitu))
        forms_out["fp32_insitu"] = o
    if d12 is not None:
        o = {"ms_per_step": d12["ms_per_step"], "value": d12["value"], "n_dirs": 12,
             "external_ms": d12["stages_ms"]["external"], "rows_ms": d12["stages_ms"]["rows"],
             "step_frac": alg_bytes_step(tin, 12) / (d12["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if ref_check12 is not None:
            o["max_rel_err_vs_oracle"] = float(np.max(np.abs(d12["sample"] - ref_check12) / ref_check12))
        forms_out[f"{args.precision}_D12"] = o
    relerr, lnerr = errs(main_form)

    dtype = {"fp32": "f32", "bf16x2": "bf16x2 (f32 accumulate)", "fp16x2": "f16x2 (f32 accumulate)"}[args.precision]
    rec = {
        "metric": "cell*directions/s of full column sweep",
        "value": value,
        "unit": "cell*dir/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{wl}, {D} {'paper M x N (3 x 4)' if sphere else 'HEALPix'} sectors, "
                               f"{args.precision} external shells + fused screening",
                   "n_leaf": tin.n_leaf, "n_dirs": D, "levels": L + 1, "precision": args.precision,
                   "step": "pyramid rebuild + column sweep"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"k_target_leaves<{D}>|adaptive {tin.n_leaf} leaves D={D}" if amr
                                                 else f"k_target_rows<{D}>|uniform {1 << L}^3 D={D}"),
                     "kernel": kname, "kernel_ms": stage_ms["rows"], "alg_bytes": step_bytes,
                     "alg_bytes_what": "per step: leaf densities read (4 B), coarse pyramid cells written once "
                                       "(4 B), rows of N (4 D B) and chi (4 B) written; the kernel's time is the "
                                       "sum of its launches in one step",
                     "step_frac": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "hbm_ceiling": hbm_ceiling(torch, tin.n_leaf * D),
        "stages_ms": stage_ms,
        "sweep": {"alg_bytes": step_bytes, "ms": stage_ms["sweep"],
                  "GB_per_s": step_bytes / (stage_ms["sweep"] * 1e-3) / 1e9},
        "forms": forms_out,
        "cpu_baseline": cpu,
        **({"sphere_test": e1} if e1 is not None else {}),
        "max_rel_err_vs_oracle_sample": relerr,
        "max_abs_dlnN_vs_oracle_sample": lnerr,
    }
    print(json.dumps(rec))


def bench_surrogate(args):
    """Learned surrogate: a network for 512^3 grids trained on seeded 256^3
    fields (each refined into 2^9 equal leaves; labels: the method's near
    shells dl = 1..3), run on an unseen 512^3 field; the timed path is the
    pyramid, inference (network near shells + the method's internal + local
    part and coarse shells) + the 1 % sampled check + fallback of the failing
    8^3 tiles, beside the plain FP32 sweep of the same field."""
    import torch

    from paper_1410_0624_amd import colden, surrogate_train, synth

    dev = torch.device("cuda:0")
    D = 12
    dirs = colden.directions(colden.CD_DIR_HEALPIX, 1)
    w = colden.Weights(dirs)
    L = 9
    t0 = time.time()
    tins = synth.workloads_uniform(8, list(range(100, 100 + args.train_fields)), sigma=1.5, mean=10.0)
    fields = [surrogate_train.label_field(t, w, L, dev) for t in tins]
    del tins
    torch.cuda.synchronize()
    t_data = time.time() - t0
    print(f"# {args.train_fields} training fields with labels in {t_data:.1f}s", file=sys.stderr, flush=True)
    nrm = surrogate_train.norms(fields)
    surr = colden.Surrogate(D, 256, colden.CD_SURR_BF16, 1, norm=nrm, leaf_level=L)
    t0 = time.time()
    log = surrogate_train.fit(surr, fields, steps=args.train_steps, batch=args.train_batch, lr=2e-3,
                              lr_final=5e-5, seed=2, log_every=max(args.train_steps // 10, 1))
    torch.cuda.synchronize()
    t_train = time.time() - t0
    print(f"# trained {args.train_steps} steps in {t_train:.1f}s, loss {log[0][1]:.4f} -> {log[-1][1]:.4f}",
          file=sys.stderr, flush=True)
    del fields
    torch.cuda.empty_cache()

    tin = synth.workload_uniform(L, sigma=1.5, mean=10.0, seed=999)
    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    tree = colden.Tree(tin, leaf, max_dirs=D)
    Np = torch.empty((tin.n_leaf, D), dtype=torch.float32, device=dev)
    chip = torch.empty(tin.n_leaf, dtype=torch.float32, device=dev)
    Ns_ = torch.empty_like(Np)
    chis = torch.empty_like(chip)
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def plain():
        tree.update(leaf)
        colden.column_densities(tree, w, Np, chip)

    fb = {}

    def surrogate():
        tree.update(leaf)
        surr.infer(tree, w, Ns_, chis)
        fb["r"] = surr.check_fallback(tree, w, Ns_, chis, frac=0.01, tol_chi=0.03, seed=7)

    def infer_only():
        tree.update(leaf)
        surr.infer(tree, w, Ns_, chis)

    ms_plain = timed(plain, max(args.steps // 5, 3))
    ms_infer = timed(infer_only, 3)
    chi_net = chis.cpu().numpy().astype(np.float64)
    ms_surr = timed(surrogate, 3)
    nfail, ntiles, emax = fb["r"]
    ref = chip.cpu().numpy().astype(np.float64)
    e_net = np.abs(chi_net - ref) / ref
    e_fin = np.abs(chis.cpu().numpy().astype(np.float64) - ref) / ref
    q = lambda e: {"mean": float(e.mean()), "p99": float(np.percentile(e, 99)), "max": float(e.max())}
    # the network runs once per level-7 cell (its leaves share the features),
    # with a block of D outputs for each of its 8 octs
    net_rows = 1 << 21
    flops = 2.0 * net_rows * (576 * 256 + 256 * 256 + 256 * surr.Dout)
    achieved = flops / (ms_infer * 1e-3) / 1e12

    cpu = None
    orc = None
    if not args.no_cpu:
        import oracle
        tr = oracle.Tree(tin)
        threads = os.cpu_count() or 1
        n1 = 1 << (L - 1)
        rng = np.random.default_rng(0)
        octs = rng.choice(n1 ** 3, size=min(args.cpu_sample_octs or int(2e8 / (8 * D)), n1 ** 3), replace=False)
        ax, ay, az = octs % n1, (octs // n1) % n1, octs // (n1 * n1)
        n = 1 << L
        tg = np.concatenate([((2 * az + (o >> 2)) * n + 2 * ay + ((o >> 1) & 1)) * n + 2 * ax + (o & 1)
                             for o in range(8)]).astype(np.int64)
        t0 = time.time()
        refc = tr.columns(dirs, tg, nthreads=threads)
        chi_o = oracle.screening(refc)
        dt = time.time() - t0
        cpu = {"value": float(tg.shape[0] * D / dt), "unit": "cell*dir/s", "cores": threads, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"{octs.shape[0]} random octs ({tg.shape[0]} leaves) of the 512^3 field, FP64 OpenMP "
                         f"oracle (the method itself), {dt:.1f} s"}
        got = chis.cpu().numpy().astype(np.float64)[tg]
        orc = q(np.abs(got - chi_o) / chi_o)

    rec = {
        "metric": "cell*directions/s of full column sweep",
        "value": tin.n_leaf * D / (ms_surr * 1e-3),
        "unit": "cell*dir/s",
        "n_gpus": 1,
        "steps": 3,
        "warmup": 1,
        "ms_per_step": ms_surr,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 (f32 accumulate)",
        "data": "synthetic",
        "config": {"workload": f"learned surrogate (MLP 576-256-256-96: near shells dl=1..3 of the 8 octs of a "
                               f"level-7 cell, bf16 on the matrix cores) trained on {args.train_fields} seeded 256^3 "
                               f"log-normal fields (sigma_ln n=1.5, mean 10 cm^-3, box 10 pc) refined to 512^3, run "
                               f"on an unseen 512^3 field (seed 999), 12 HEALPix sectors; step = pyramid + inference "
                               f"(+ the method's internal/local and dl>=4 parts) + 1% sampled check per 8^3 tile + "
                               f"fallback (tol 3% in chi)",
                   "n_leaf": tin.n_leaf, "n_dirs": D},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": achieved / 2500.0, "traffic": None,
                     "kernel": "inference (features + network on 2^21 level-7 rows + coarse tables + row kernel)",
                     "kernel_ms": ms_infer, "flops_per_launch": flops, "network_rows": net_rows},
        "forms": {"plain_fp32": {"ms_per_step": ms_plain, "value": tin.n_leaf * D / (ms_plain * 1e-3)},
                  "surrogate_infer_only": {"ms": ms_infer, "chi_rel_err_vs_plain": q(e_net)},
                  "surrogate_with_fallback": {"ms": ms_surr, "speedup_vs_plain": ms_plain / ms_surr,
                                              "fallback_tiles": nfail, "tiles": ntiles,
                                              "fallback_fraction": nfail / ntiles,
                                              "max_sampled_chi_err": emax,
                                              "chi_rel_err_vs_plain": q(e_fin),
                                              "chi_rel_err_vs_oracle_sample": orc}},
        "training": {"fields": args.train_fields, "steps": args.train_steps, "batch": args.train_batch,
                     "seconds": t_train, "label_seconds": t_data, "loss_log": log},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
