#!/usr/bin/env python3
"""Benchmark of the C* Pfaffian-sign hot path on one MI355X.

One step = one block application of the Wilson-clover operator D to 16
right-hand sides at 16 masses of the kappa path, in the solver's inner form
(FP32 spinors and arithmetic, BF16-stored links), on the batched 32^4 field,
in a single launch.  Inputs are resident in HBM before the timed region; the
launches are timed with HIP events on the handle's stream and the steps with
the wall clock between device synchronisations.

After the timed steps, on the same field: the single-RHS apply in every
precision, the CPU oracle on a bounded sample, and the time to sign over the
32-point kappa path for the mixed-precision, plain FP64 and learned forms,
and for the mixed form in the paper's order (step A upward from the target
with lambda_bar by the power method on Q^-2, then step B); then the
mass-reweighting rows (the even-odd apply, log W_eo, one W_mass estimate,
lambda_bar by the power method, the ensemble driver on 16^4 fields) --
each only while the wall-clock budget allows (skipped legs are named in the
output).

Printed: ONE JSON line -- RHS-applies/s of the block step, the roofline of
its kernel (algorithmic bytes over the HIP-event launch time), the CPU oracle,
the seconds per Pfaffian sign and the mass-reweighting measurements.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
T_START = time.time()

# sources of the apply kernels; the committed counter summary records their hash
APPLY_SOURCES = ("paper_2108_11989_amd/csrc/kernels_dirac.hip", "paper_2108_11989_amd/csrc/lattice_dev.h",
                 "paper_2108_11989_amd/csrc/stencil_dev.h", "paper_2108_11989_amd/csrc/tune.cpp")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "apply_traffic_32x32x32x32.md")


def apply_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in APPLY_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(prec_name: str, rhs_per_launch: int):
    """HBM bytes per launch of the block step's kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE runs of this bench,
    each scaled by what the counter reads for a plain copy of known size):
    the line `traffic <form> <nrhs> <bytes>`; None if the summary is missing,
    has no line for this launch, or was taken on other kernel sources."""
    try:
        lines = open(TRAFFIC_SUMMARY).read().splitlines()
    except OSError:
        return None
    src = [ln.split()[-1] for ln in lines if ln.startswith("source_sha256:")]
    if not src or src[0] != apply_source_hash():
        return None
    for ln in lines:
        f = ln.split()
        if len(f) == 4 and f[0] == "traffic" and f[1] == prec_name and int(f[2]) == int(rhs_per_launch):
            return float(f[3])
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(prec: int, nsites2: int, launches: int, rhs: int, operands: int = 0) -> float:
    """Minimum HBM bytes of the apply launches (per doubled site, per launch):
    every input spinor read once, every output written once, links and clover
    read once per physical site (shared by its conjugate copy), and every
    extra vector of a fused epilogue (out = a D in + b y + c z) read once:
      FP64: 384 B per RHS + (4 links x 144 B + clover 576 B)/2, 192 B per operand
      FP32: 192 B per RHS + (4 x (48 B rows + 8 B phase) + clover 288 B)/2, 96 B per operand
      FP32 + BF16 links: 192 B per RHS + (4 x (24 B rows + 8 B phase) + 288 B)/2, 96 B per operand
    """
    per_rhs, shared = {0: (384.0, 576.0), 1: (192.0, 256.0), 2: (192.0, 208.0)}[prec]
    return nsites2 * (per_rhs * rhs + shared * launches + per_rhs / 2 * operands)


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(su3, th, q, T, L, budget_s=20.0):
    """The oracle's FP64 apply of Q timed on the host cores (bounded sample).
    The oracle's setup (field strength and link table, once per operator) is
    not counted; applies run until about half the budget is spent, at most 20."""
    import numpy as np

    from oracle import dirac as odirac
    from paper_2108_11989_amd import synth
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    t0 = time.time()
    op = odirac.Operator(su3, th, q)
    op.links()
    t_setup = time.time() - t0
    psi = synth.random_spinor(T, L, 5)
    n = 0
    t0 = time.time()
    while True:
        psi = op.apply(psi, -0.3, True)
        psi /= np.linalg.norm(psi)
        n += 1
        if time.time() - t0 > budget_s * 0.5 or n >= 20:
            break
    dt = time.time() - t0
    return {"value": n / dt, "unit": "Dirac applies/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "threads": threads, "host_cpus": len(os.sched_getaffinity(0)),
            "sample": f"{n} FP64 oracle applies of Q at {T}x{L}^3 (one RHS each; setup of the field strength "
                      f"and link table, {t_setup:.1f} s, not counted)"}


def cpu_other_configs(budget_s=30.0):
    """The oracle beside the GPU at the other sizes (bounded samples): FP64
    applies of Q per second at the single-vector 16^4 and the paper-scale
    64x32^3 workloads, and the whole sign over the tiny workload's 16-point
    kappa path by dense inertia on the host against pfaffian_sign on the GPU
    (each sign at one mass, by the same path)."""
    import numpy as np
    import torch

    from oracle import dirac as odirac
    from oracle import sign as osign
    from paper_2108_11989_amd import cstar, synth
    out = {}
    for name, n_max in (("single_16^4", 40), ("paper_64x32^3", 6)):
        w = synth.WORKLOADS[name]
        T, L = w["T"], w["L"]
        su3, th = synth.make_field(T, L, w["eps"], w["seed"], smear_steps=w["smear"], exp_backend="torch")
        op = odirac.Operator(su3, th, w["q"][-1])
        op.links()
        psi = synth.random_spinor(T, L, 5)
        n, t0 = 0, time.time()
        while n < n_max and time.time() - t0 < budget_s / 4:
            psi = op.apply(psi, -0.3, True)
            psi /= np.linalg.norm(psi)
            n += 1
        dt = time.time() - t0
        out[name] = {"applies_per_s": n / dt, "sample": f"{n} FP64 oracle applies of Q at {T}x{L}^3"}
        del op, su3, th, psi
    w = synth.WORKLOADS["tiny_4x2^3"]
    su3, th = synth.make_field(w["T"], w["L"], w["eps"], w["seed"])
    q = w["q"][0]
    path = np.asarray(synth.kappa_to_m0(w["kappas"]), dtype=np.float64)
    op = odirac.Operator(su3, th, q)
    t0 = time.time()
    ref = [osign.sign_inertia(op, float(m)) for m in path]
    t_cpu = time.time() - t0
    g = cstar.Gauge(su3, th, q, synth.CSW_SU3, synth.CSW_U1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sg, rep = g.pfaffian_sign(path, k=4, eig=cstar.eig_opts(tol=1e-10))
    t_gpu = time.perf_counter() - t0
    g.close()
    out["tiny_4x2^3_sign"] = {"cpu_dense_inertia_s": t_cpu, "gpu_pfaffian_sign_s": t_gpu,
                              "agree": bool(np.array_equal(np.asarray(sg), np.asarray(ref))),
                              "signs": "".join("+" if v > 0 else "-" for v in ref)}
    return out


def train_network(args, w, q, m_train):
    """The learned preconditioner, trained here on the GPU (library kernels) on
    smoothed 8^4 fields of the workload's distribution (the network is local:
    its weights do not depend on the lattice size)."""
    from paper_2108_11989_amd import cstar, learned, synth
    t0 = time.perf_counter()
    gs, xs = [], []
    for i in range(args.train_fields):
        s3, t3 = synth.make_field(8, 8, w["eps"], 5000 + i, smear_steps=w["smear"])
        g = cstar.Gauge(s3, t3, q, synth.CSW_SU3, synth.CSW_U1)
        gs.append(g)
        xs.append(learned.training_vectors(g, m_train, 4, 4, seed=7000 + 10 * i))
    t_data = time.perf_counter() - t0
    net, hist = learned.train(gs, xs, 8, m_train, args.train_epochs, 1e-3)
    for g in gs:
        g.close()
    info = {"fields": args.train_fields, "lattice": "8x8^3", "epochs": args.train_epochs, "pairs_per_field": 8,
            "loss_first": float(hist[0]), "loss_last": float(hist[-1]), "s_data": t_data,
            "s_train": time.perf_counter() - t0 - t_data}
    log(f"[bench] network trained: loss {hist[0]:.4f} -> {hist[-1]:.4f} ({info['s_train']:.1f} s)")
    return net, info


FORMS = (("plain_fp64", "fp64", 0), ("plain_mixed", "bf16", 0), ("learned_mixed", "bf16", 1))


def compare_lambda_bar(args, su3_d, th_d, q, masses):
    """lambda_bar by the power method with Chebyshev acceleration on Q^-2 (the
    paper's step-A solver) against the block eigensolver at the same relative
    accuracy, cold at each mass: seconds, D applies, the two values.  The block
    solver runs with the bench's k (a block of 2k + max(8, k) vectors): a
    smaller block cannot hold the smooth fields' near-degenerate low multiplets
    of Q^2 and converges very slowly."""
    import numpy as np
    import torch

    from paper_2108_11989_amd import cstar, synth
    out = []
    for m in masses:
        g = cstar.Gauge(su3_d, th_d, q, synth.CSW_SU3, synth.CSW_U1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, bound, st = g.lambda_bar_power(float(m), tol=args.lbar_tol, max_outer=args.lbar_max_outer,
                                            raise_on_noconv=False, inner=cstar.FP32_BF16LINKS)
        t_pow = time.perf_counter() - t0
        conv = bound <= args.lbar_tol * lam
        g.close()
        log(f"[bench] lambda_bar at m0={float(m):+.4f}: power {lam:.6f} +- {bound:.1e} in {t_pow:.1f} s "
            f"({st.applies_inner} mixed + {st.applies_fp64} FP64 applies, {st.solves} solves, converged {conv})")
        g = cstar.Gauge(su3_d, th_d, q, synth.CSW_SU3, synth.CSW_U1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, res, st2 = g.lowest_eigs(float(m), args.k, cstar.eig_opts(inner=cstar.FP32_BF16LINKS,
                                                                      tol=args.lbar_tol, max_iter=1000))
        t_blk = time.perf_counter() - t0
        g.close()
        r = {"m0": float(m),
             "power": {"lambda_bar": lam, "half_width": bound, "converged": bool(conv), "s": t_pow,
                       "outer": st.outer, "solves": st.solves, "cg_iterations": st.cg_iterations,
                       "applies_fp64": st.applies_fp64, "applies_inner": st.applies_inner},
             "block": {"k": args.k, "lambda_bar": float(abs(ev[0])), "resid": float(res[0]), "s": t_blk,
                          "iterations": st2.iterations, "applies_inner": st2.applies_inner,
                          "applies_fp64": st2.applies_fp64},
             "agree": bool(abs(lam - abs(ev[0])) <= bound + float(res[0]))}
        out.append(r)
        log(f"[bench] lambda_bar at m0={float(m):+.4f}: block k={args.k} {abs(ev[0]):.6f} +- {res[0]:.1e} in "
            f"{t_blk:.1f} s ({st2.applies_inner} + {st2.applies_fp64} applies), agree {r['agree']}")
    return out


def compare_forms(args, net, su3_d, th_d, q, masses, full_path):
    """Plain FP64, plain mixed precision and learned + mixed precision: seconds
    and applies per eigensolve at the given masses (cold start), or per
    Pfaffian sign over the whole path."""
    import numpy as np
    import torch

    from paper_2108_11989_amd import cstar, synth
    inner = {"bf16": cstar.FP32_BF16LINKS, "fp64": cstar.FP64}
    res = {}
    for name, prec, use_nn in FORMS:
        g = cstar.Gauge(su3_d, th_d, q, synth.CSW_SU3, synth.CSW_U1)
        if use_nn:
            net.attach(g)
        opts = cstar.eig_opts(inner=inner[prec], tol=args.tol, max_iter=1000, use_nn=use_nn)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if full_path:
            signs, rep = g.pfaffian_sign(masses, k=args.k, eig=opts)
            r = {"s_per_sign": time.perf_counter() - t0, "applies": rep.applies, "nn_applies": rep.nn_applies,
                 "fallbacks": rep.nn_fallbacks, "points_solved": rep.n_points,
                 "signs": "".join("+" if v > 0 else "-" for v in signs)}
        else:
            r = {"solves": []}
            for m in masses:
                t1 = time.perf_counter()
                ev, res_, st = g.lowest_eigs(float(m), args.k, opts)
                r["solves"].append({"m0": float(m), "s": time.perf_counter() - t1, "iterations": st.iterations,
                                    "applies_inner": st.applies_inner, "applies_fp64": st.applies_fp64,
                                    "nn_applies": st.nn_applies, "fallback": st.nn_fallback,
                                    "lambda": [float(x) for x in ev], "resid_max": float(np.max(res_))})
            r["s"] = time.perf_counter() - t0
        if use_nn:
            cstar.Net.detach(g)
        g.close()
        res[name] = r
        log(f"[bench] {name}: {json.dumps(r)[:300]}")
    if full_path:
        res["signs_agree"] = len({res[n]["signs"] for n, _, _ in FORMS}) == 1
    else:
        # the plain FP64 solve judges the others: |lambda - lambda_fp64| within the residual bounds
        ref = res["plain_fp64"]["solves"]
        res["eigenvalues_agree"] = all(
            abs(a - b) <= sa["resid_max"] + sb["resid_max"] + 1e-12
            for n in ("plain_mixed", "learned_mixed")
            for sa, sb in zip(res[n]["solves"], ref) for a, b in zip(sa["lambda"], sb["lambda"]))
    return res


def kernel_probe(args, su3_d, th_d, q, T, L):
    """Time the apply kernels alone (single RHS in every precision, and the
    solver's multi-RHS block in the inner precision) with HIP events."""
    import torch

    from paper_2108_11989_amd import cstar, synth
    g = cstar.Gauge(su3_d, th_d, q, synth.CSW_SU3, synth.CSW_U1)
    nsites2 = 2 * T * L ** 3
    nb = args.probe_nrhs or (2 * args.k + max(8, args.k))
    res = {}
    for prec, name in [(cstar.FP64, "fp64"), (cstar.FP32, "fp32"), (cstar.FP32_BF16LINKS, "bf16")]:
        for nrhs in (1, nb):
            nin, nout = g.new_native(nrhs, prec), g.new_native(nrhs, prec)
            nin.normal_()
            masses = [-0.3] * nrhs
            for _ in range(2):
                g.apply(nin, nout, masses, prec, True)
            g.timing(True)
            for _ in range(args.probe_reps):
                g.apply(nin, nout, masses, prec, True)
            tm = g.read_timing()[prec]
            g.timing(False)
            avg = tm["ms"] / tm["launches"]
            gbs = algorithmic_bytes(prec, nsites2, tm["launches"], tm["rhs"]) / (tm["ms"] * 1e-3) / 1e9
            res[f"{name}_x{nrhs}"] = {"avg_ms": avg, "GBs": gbs, "applies_per_s": nrhs / (avg * 1e-3)}
            log(f"[probe] {name} nrhs={nrhs}: {avg:.4f} ms/launch, {nrhs / (avg * 1e-3):.0f} applies/s, "
                f"{gbs:.0f} GB/s algorithmic ({100 * gbs / HBM_PEAK_GBS:.1f}% of 8 TB/s)")
            del nin, nout
    if args.copy_probe_gib > 0:
        n = int(args.copy_probe_gib * (1 << 30) // 4)
        a = torch.empty(n, dtype=torch.float32, device="cuda")
        a.fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # blit copy
        torch.mul(a, 1.0, out=b)  # elementwise kernel: 16-byte vector loads per lane, like the apply kernels
        torch.cuda.synchronize()
        log(f"[probe] device copy (blit and elementwise) of {n * 4} bytes done")
    g.close()
    print(json.dumps({"kernel_probe": res, "lattice": f"{T}x{L}^3"}), flush=True)


def block_step_masses(kappas, nrhs):
    """nrhs masses spread over the kappa path (every other point of the 32-point path for 16)."""
    import numpy as np

    from paper_2108_11989_amd import synth
    idx = np.linspace(0, len(kappas) - 1, nrhs).round().astype(int)
    return [float(m) for m in synth.kappa_to_m0(np.asarray(kappas)[idx])]


def single_rhs_rates(g, nsites2, reps=20):
    """Single-RHS apply of Q in every precision on the step's field (HIP events)."""
    from paper_2108_11989_amd import cstar
    out = {}
    for prec, name in [(cstar.FP64, "fp64"), (cstar.FP32, "fp32"), (cstar.FP32_BF16LINKS, "fp32_bf16links")]:
        nin, nout = g.new_native(1, prec), g.new_native(1, prec)
        nin.normal_()
        for _ in range(3):
            g.apply(nin, nout, [-0.3], prec, True)
        g.timing(True)
        for _ in range(reps):
            g.apply(nin, nout, [-0.3], prec, True)
        tm = g.read_timing()[prec]
        g.timing(False)
        ms = tm["ms"] / tm["launches"]
        gbs = algorithmic_bytes(prec, nsites2, 1, 1) / (ms * 1e-3) / 1e9
        out[name] = {"ms": ms, "applies_per_s": 1e3 / ms, "GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
        del nin, nout
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batched_32^4")
    ap.add_argument("--nrhs", type=int, default=16, help="right-hand sides (and masses) of the block step")
    ap.add_argument("--budget-s", type=float, default=480.0,
                    help="wall-clock budget from process start; optional legs that would exceed it are skipped")
    ap.add_argument("--legs", default="single,cpu,mixed,fp64,learned,stepa,reweight",
                    help="legs after the timed steps (comma list of single, cpu, mixed, fp64, learned, resid, stepa, "
                         "reweight; 'none')")
    ap.add_argument("--k", type=int, default=4, help="eigenvalues (Kramers pairs) per mass point")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--block", type=int, default=0, help="eigensolver block size (0: 2k + max(8, k))")
    ap.add_argument("--path-points", type=int, default=0, help="use only the first n kappas (0 = all)")
    ap.add_argument("--kernel-probe", action="store_true",
                    help="only time the apply kernels on the workload lattice (for profiler runs)")
    ap.add_argument("--probe-reps", type=int, default=20)
    ap.add_argument("--probe-nrhs", type=int, default=0, help="multi-RHS width of the probe (0: the solver block)")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="also run one device copy of this many GiB (counter calibration)")
    ap.add_argument("--compare-path", action="store_true",
                    help="learned vs plain over the whole path (three Pfaffian signs; minutes), instead of the timed step")
    ap.add_argument("--compare-lbar", type=int, default=0,
                    help="power method on Q^-2 vs the block eigensolver for lambda_bar at the first n path masses, "
                         "instead of the timed step")
    ap.add_argument("--lbar-tol", type=float, default=1e-3, help="relative accuracy of lambda_bar in --compare-lbar")
    ap.add_argument("--lbar-max-outer", type=int, default=100)
    ap.add_argument("--sign-path", action="store_true",
                    help="instead of the block step: Pfaffian signs over the path for every charge of the workload "
                         "(--learned: with the trained preconditioner), timed")
    ap.add_argument("--inner", default="bf16", choices=["bf16", "fp32", "fp64"], help="filter precision of --sign-path")
    ap.add_argument("--learned", action="store_true", help="--sign-path with the learned preconditioner")
    ap.add_argument("--charges", default="", help="comma-separated indices of the workload's quark charges (default: all)")
    ap.add_argument("--fp64-rerun", action="store_true",
                    help="instead of the block step: eigenvalues at --rerun-masses path masses in FP64, mixed and "
                         "learned forms, errors against FP64 (charge index --charges, default 0)")
    ap.add_argument("--rerun-masses", type=int, default=4)
    ap.add_argument("--rerun-signs", action="store_true", help="with --fp64-rerun: also the sign over the path "
                                                               "in FP64 and mixed precision")
    ap.add_argument("--c3-train", default="",
                    help="instead of the block step: train the network on --c3-fields fields of the workload's "
                         "distribution (seeds 1000.., 4 plain-solver low modes + 4 Gaussian vectors each, streamed, "
                         "--c3-steps Adam steps per field) and save its FP32 weights (.npy) to this path")
    ap.add_argument("--c3-eval", default="",
                    help="instead of the block step: weights (.npy) to judge on --c3-test held-out fields (seeds "
                         "2000..): plain vs learned mixed-precision eigensolves at the lightest path mass, and the "
                         "sign over the path on the first of them")
    ap.add_argument("--reweight-probe", action="store_true",
                    help="instead of the block step: the even-odd apply timed in every form (HIP events), W_eo, "
                         "one W_mass estimate, lambda_bar by the power method and the ensemble driver, at the "
                         "workload's size (the ensemble on 16^4 fields of its distribution)")
    ap.add_argument("--ensemble-probe", type=int, default=0,
                    help="instead of the block step: W_sgn by the ensemble driver over this many fields of the "
                         "workload's distribution and size (seeds 3000..), flavours q = 2/3 and -1/3, at the "
                         "lightest path mass")
    ap.add_argument("--c3-fields", type=int, default=64)
    ap.add_argument("--c3-steps", type=int, default=3)
    ap.add_argument("--c3-test", type=int, default=8)
    ap.add_argument("--c3-sign", type=int, default=1, help="with --c3-eval: 0 skips the signs")
    ap.add_argument("--train-fields", type=int, default=8)
    ap.add_argument("--train-epochs", type=int, default=30)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path in this library "
              "(an ensemble shards by configuration and flavour with no exchange; a single lattice would be cut "
              "along t with one halo exchange per apply).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2108_11989_amd import cstar, synth

    if not torch.cuda.is_available():
        log("no GPU")
        sys.exit(1)
    w = synth.WORKLOADS[args.workload]
    T, L, q = w["T"], w["L"], w["q"][0]
    if args.c3_train or args.c3_eval:
        c3(args, w)
        return
    if args.ensemble_probe > 0:
        ensemble_probe(args, w)
        return
    log(f"[bench] workload {args.workload}: {T}x{L}^3, eps {w['eps']}, seed {w['seed']}, smear {w['smear']}")
    t0 = time.time()
    su3, th = synth.make_field(T, L, w["eps"], w["seed"], smear_steps=w["smear"], smear_backend="torch")
    log(f"[bench] field generated in {time.time() - t0:.1f} s")
    su3_d = torch.from_numpy(su3).cuda().contiguous()
    th_d = torch.from_numpy(th).cuda().contiguous()
    if args.kernel_probe:
        kernel_probe(args, su3_d, th_d, q, T, L)
        return
    kappas = w["kappas"] if args.path_points <= 0 else w["kappas"][: args.path_points]
    path = np.asarray(synth.kappa_to_m0(kappas), dtype=np.float64)
    nsites2 = 2 * T * L ** 3

    if args.compare_path:
        net, info = train_network(args, w, q, float(path[0]))
        res = compare_forms(args, net, su3_d, th_d, q, path, True)
        net.close()
        print(json.dumps({"learned_vs_plain_path": res, "train": info, "workload": args.workload,
                          "kappa_points": int(len(path)), "k_pairs": args.k, "eig_tol": args.tol}), flush=True)
        return
    if args.compare_lbar > 0:
        res = compare_lambda_bar(args, su3_d, th_d, q, path[:args.compare_lbar])
        print(json.dumps({"lambda_bar_power_vs_block": res, "workload": args.workload, "tol": args.lbar_tol}),
              flush=True)
        return
    if args.sign_path:
        sign_path(args, w, su3_d, th_d, path, nsites2)
        return
    if args.fp64_rerun:
        fp64_rerun(args, w, su3_d, th_d, path)
        return
    if args.reweight_probe:
        reweight_probe(args, w, su3_d, th_d, path)
        return

    # ---------------------------------------------------------------- the timed block step
    prec = cstar.FP32_BF16LINKS
    g = cstar.Gauge(su3_d, th_d, q, synth.CSW_SU3, synth.CSW_U1)
    masses = block_step_masses(kappas, args.nrhs)
    nin, nout = g.new_native(args.nrhs, prec), g.new_native(args.nrhs, prec)
    torch.manual_seed(0)
    nin.normal_()
    log(f"[bench] block step: {args.nrhs} right-hand sides at masses {masses[0]:+.4f} .. {masses[-1]:+.4f}")
    for _ in range(args.warmup):
        g.apply(nin, nout, masses, prec, False)
    torch.cuda.synchronize()
    g.timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.apply(nin, nout, masses, prec, False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = g.read_timing()[prec]
    g.timing(False)
    avg_ms = tm["ms"] / max(tm["launches"], 1)
    byts = algorithmic_bytes(prec, nsites2, 1, args.nrhs)
    achieved = byts / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic("bf16", args.nrhs) if args.workload == "batched_32^4" else None
    log(f"[bench] {args.steps} steps in {dt * 1e3:.2f} ms; kernel {avg_ms:.3f} ms per launch (HIP events), "
        f"{achieved:.0f} GB/s algorithmic ({100 * achieved / HBM_PEAK_GBS:.1f} % of 8 TB/s)")
    # after the timed region: 50 launches, each between two HIP events on the
    # handle's stream (the null stream, torch's current one), for the spread
    launch_ms = None
    cur = torch.cuda.current_stream()
    if cur.cuda_stream == 0:
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(50)]
        for e0, e1 in evs:
            e0.record(cur)
            g.apply(nin, nout, masses, prec, False)
            e1.record(cur)
        torch.cuda.synchronize()
        per = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
        launch_ms = {"n": len(per), "median": per[len(per) // 2], "min": per[0], "max": per[-1]}
        log(f"[bench] 50 launches one by one: median {launch_ms['median']:.3f} ms, min {launch_ms['min']:.3f} ms")
    del nin, nout

    legs = set() if args.legs == "none" else set(args.legs.split(","))
    skipped = []

    def have(est_s, name):
        left = args.budget_s - (time.time() - T_START)
        if est_s > left:
            skipped.append(f"{name} (estimated {est_s:.0f} s, {max(left, 0):.0f} s of budget left)")
            log(f"[bench] skipping {name}: estimated {est_s:.0f} s, {left:.0f} s left")
            return False
        return True

    single = None
    if "single" in legs and have(5, "single"):
        single = single_rhs_rates(g, nsites2)
        for k_, v in single.items():
            log(f"[bench] single RHS {k_}: {v['ms']:.3f} ms, {v['GBs']:.0f} GB/s ({100 * v['frac']:.1f} %)")
    g.close()

    cpu = None
    if "cpu" in legs and have(60, "cpu"):
        log("[bench] timing the CPU oracle")
        cpu = cpu_baseline(su3, th, q, T, L)
        log(f"[bench] CPU oracle: {cpu['value']:.2f} applies/s on {cpu['threads']} threads ({cpu['cpu_model']})")
        if have(90, "cpu_other_configs"):
            cpu["other_configs"] = cpu_other_configs()
            oc = cpu["other_configs"]
            log(f"[bench] CPU oracle: {oc['single_16^4']['applies_per_s']:.1f} applies/s at 16^4, "
                f"{oc['paper_64x32^3']['applies_per_s']:.2f} at 64x32^3; tiny sign path: dense inertia "
                f"{oc['tiny_4x2^3_sign']['cpu_dense_inertia_s']:.2f} s, GPU "
                f"{oc['tiny_4x2^3_sign']['gpu_pfaffian_sign_s']:.2f} s, agree {oc['tiny_4x2^3_sign']['agree']}")

    # ---------------------------------------------------------------- time to sign, three forms
    signs = {}
    inner = {"bf16": cstar.FP32_BF16LINKS, "fp64": cstar.FP64}

    def one_sign(name, form, net=None, step_a=False, resid=False):
        gg = cstar.Gauge(su3_d, th_d, q, synth.CSW_SU3, synth.CSW_U1)
        if net is not None:
            net.attach(gg)
        opts = cstar.eig_opts(inner=inner[form], tol=args.tol, max_iter=1000,
                              use_nn=2 if resid else int(net is not None), block=args.block)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sg, rep = gg.pfaffian_sign(path, k=args.k, eig=opts, step_a_power=step_a)
        s_ = time.perf_counter() - t1
        gg.close()
        signs[name] = {"s_per_sign": s_, "applies": rep.applies, "mass_points_solved": rep.n_points,
                       "crossings": rep.n_crossings, "nn_applies": rep.nn_applies, "nn_fallbacks": rep.nn_fallbacks,
                       "signs": "".join("+" if v > 0 else "-" for v in sg)}
        log(f"[bench] sign {name}: {s_:.1f} s, {rep.n_points} points solved, {rep.applies} applies, "
            f"signs {signs[name]['signs']}")
        return s_

    s_mixed = 60.0
    if "mixed" in legs and have(90, "sign mixed"):
        s_mixed = one_sign("mixed", "bf16")
    if "fp64" in legs and have(2.2 * s_mixed + 10, "sign plain_fp64"):
        one_sign("plain_fp64", "fp64")
    if "learned" in legs and have(1.4 * s_mixed + 40, "sign learned_mixed"):
        net, info = train_network(args, w, q, float(path[0]))
        one_sign("learned_mixed", "bf16", net)
        signs["learned_mixed"]["train"] = info
        net.close()
        shipped = os.path.join(os.path.dirname(os.path.abspath(cstar.__file__)), "nn_c3_32x32x32x32.npy")
        if args.workload == "batched_32^4" and os.path.exists(shipped) and have(1.4 * s_mixed + 10,
                                                                                 "sign learned_c3_mixed"):
            # the network trained at this workload's size on 64 fields of its distribution
            net = cstar.Net(np.load(shipped, allow_pickle=False).astype(np.float32))
            one_sign("learned_c3_mixed", "bf16", net)
            signs["learned_c3_mixed"]["weights"] = "nn_c3_32x32x32x32.npy (64 fields at 32^4, 3 Adam steps each)"
            net.close()
    if "resid" in legs and have(1.2 * s_mixed + 10, "sign mixed_resid"):
        # the same extra directions as the learned form with M = 1: the residuals themselves
        one_sign("mixed_resid", "bf16", resid=True)
    if "stepa" in legs and have(1.5 * s_mixed + 30, "sign mixed_step_a"):
        # the paper's order: step A upward from the target with lambda_bar by the power method
        # on Q^-2, the block solver only above where step A stops
        one_sign("mixed_step_a", "bf16", step_a=True)
    if len({v["signs"] for v in signs.values()}) > 1:
        log("[bench] WARNING: the forms disagree on the signs")
    reweight = None
    if "reweight" in legs and have(60, "reweight"):
        # even-odd apply, W_eo, W_mass, lambda_bar by the power method, the ensemble driver
        reweight = reweight_rows(args, w, su3_d, th_d, path)

    out = {
        "metric": "Dirac applies/s & HBM GB/s (% peak) at 32^4; s per Pfaffian sign, learned vs plain",
        "value": args.nrhs * args.steps / dt,
        "unit": "Dirac applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 (bf16-stored links)",
        "data": "synthetic",
        "config": {"workload": args.workload, "lattice": f"{T}x{L}^3", "sites_doubled": nsites2,
                   "step": f"one launch: D applied to {args.nrhs} right-hand sides at {args.nrhs} masses",
                   "nrhs": args.nrhs, "masses": masses, "charge": q,
                   "sign_path": {"kappa_points": int(len(path)), "k_pairs": args.k, "eig_tol": args.tol}},
        "roofline": {"bound": "hbm", "kernel": "k_apply_march (FP32, BF16 links, multi-RHS)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": byts, "avg_launch_ms": avg_ms},
        "launch_ms": launch_ms,
        "cpu_baseline": cpu,
        "single_rhs": single,
        "s_per_sign": {k_: v["s_per_sign"] for k_, v in signs.items()},
        "signs": signs,
        "signs_agree": len({v["signs"] for v in signs.values()}) <= 1,
        "mass_reweighting": reweight,
        "skipped": skipped,
        "wall_s": time.time() - T_START,
    }
    print(json.dumps(out), flush=True)


def fp64_rerun(args, w, su3_d, th_d, path):
    """The FP64 GPU rerun as judge: the k lowest eigenvalues at a few masses of
    the path, solved cold in plain FP64, mixed precision and learned + mixed
    (network trained on small fields of the workload's distribution), with the
    error of each form's eigenvalues against the FP64 solve; then, with
    --rerun-signs, the sign over the whole path in FP64 and in mixed precision."""
    import numpy as np
    import torch

    from paper_2108_11989_amd import cstar, synth
    q = float(w["q"][int(args.charges or 0)])
    idx = np.linspace(0, len(path) - 1, args.rerun_masses).round().astype(int)
    net, info = train_network(args, w, q, float(path[0]))
    out = {"workload": args.workload, "q": q, "k": args.k, "tol": args.tol, "masses": [], "train": info}
    forms = (("fp64", cstar.FP64, 0), ("mixed", cstar.FP32_BF16LINKS, 0), ("learned_mixed", cstar.FP32_BF16LINKS, 1))
    for i in idx:
        m = float(path[i])
        row = {"m0": m}
        for name, prec, nn in forms:
            g = cstar.Gauge(su3_d, th_d, q, synth.CSW_SU3, synth.CSW_U1)
            if nn:
                net.attach(g)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev, res, st = g.lowest_eigs(m, args.k, cstar.eig_opts(inner=prec, tol=args.tol, max_iter=1000, use_nn=nn))
            row[name] = {"lambda": [float(x) for x in ev], "resid": [float(x) for x in res],
                         "s": time.perf_counter() - t0, "applies": st.applies_inner + st.applies_fp64}
            if nn:
                cstar.Net.detach(g)
            g.close()
        ref = np.array(row["fp64"]["lambda"])
        for name in ("mixed", "learned_mixed"):
            row[name]["max_rel_err_vs_fp64"] = float(np.max(np.abs(np.array(row[name]["lambda"]) - ref) / np.abs(ref)))
        log(f"[bench] rerun m0={m:+.4f}: fp64 {row['fp64']['s']:.1f} s, mixed {row['mixed']['s']:.1f} s "
            f"(rel err {row['mixed']['max_rel_err_vs_fp64']:.1e}), learned {row['learned_mixed']['s']:.1f} s "
            f"(rel err {row['learned_mixed']['max_rel_err_vs_fp64']:.1e})")
        out["masses"].append(row)
    net.close()
    if args.rerun_signs:
        out["signs"] = {}
        for name, prec in (("mixed", cstar.FP32_BF16LINKS), ("fp64", cstar.FP64)):
            g = cstar.Gauge(su3_d, th_d, q, synth.CSW_SU3, synth.CSW_U1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sg, rep = g.pfaffian_sign(path, k=args.k, eig=cstar.eig_opts(inner=prec, tol=args.tol, max_iter=1000))
            out["signs"][name] = {"s": time.perf_counter() - t0, "signs": "".join("+" if v > 0 else "-" for v in sg),
                                  "mass_points_solved": rep.n_points, "applies": rep.applies}
            g.close()
            log(f"[bench] rerun sign {name}: {out['signs'][name]['s']:.1f} s, {out['signs'][name]['signs']}")
        out["signs_agree"] = len({v["signs"] for v in out["signs"].values()}) == 1
    print(json.dumps({"fp64_rerun": out}), flush=True)


def eo_algorithmic_bytes(prec: int, nsites2: int, nrhs: int) -> float:
    """Minimum HBM bytes of one application of D_hat = D_ee - D_eo D_oo^-1 D_oe
    in its two passes, per site of the doubled lattice (half of them even):
    per RHS the even input read by both passes, the odd intermediate written
    and read, the even output written (five half vectors); the links read by
    both passes and the odd inverse and even clover blocks once (shared by a
    site and its conjugate copy):
      FP64:             5 x 192/2 B per RHS + 2 x (4 x 144)/2 B + 576/2 B
      FP32 rows:        5 x  96/2 B per RHS + 2 x (4 x  56)/2 B + 288/2 B
      FP32 + BF16 rows: 5 x  96/2 B per RHS + 2 x (4 x  32)/2 B + 288/2 B"""
    spin = {0: 192.0, 1: 96.0, 2: 96.0}[prec]
    links = {0: 4 * 144.0, 1: 4 * 56.0, 2: 4 * 32.0}[prec]
    clov = {0: 576.0, 1: 288.0, 2: 288.0}[prec]
    return nsites2 * (5 * spin / 2 * nrhs + 2 * links / 2 + clov / 2)


def reweight_probe(args, w, su3_d, th_d, path):
    """The mass-reweighting rows measured (reweight_rows), as one JSON line."""
    print(json.dumps({"reweight_probe": reweight_rows(args, w, su3_d, th_d, path)}), flush=True)


def reweight_rows(args, w, su3_d, th_d, path):
    """Measurements of the mass-reweighting rows at the workload's size: the
    even-odd apply (HIP events; bytes as eo_algorithmic_bytes), log W_eo, one
    W_mass estimate (one Gaussian source, order-8 rational approximation),
    lambda_bar by the power method against the block solver at the lightest
    mass, and the ensemble driver on 16^4 fields of the same distribution."""
    import numpy as np
    import torch

    from paper_2108_11989_amd import cstar, synth
    T, L, q = w["T"], w["L"], w["q"][0]
    nsites2 = 2 * T * L ** 3
    m = float(path[0])
    g = cstar.Gauge(su3_d, th_d, q, synth.CSW_SU3, synth.CSW_U1)
    out = {"workload": args.workload, "lattice": f"{T}x{L}^3", "q": q, "m0": m, "eo_apply": {}}
    stream = torch.cuda.current_stream()
    for prec, name in ((cstar.FP64, "fp64"), (cstar.FP32, "fp32"), (cstar.FP32_BF16LINKS, "bf16")):
        for nrhs in (1, 16):
            a, b = g.new_native(nrhs, prec), g.new_native(nrhs, prec)
            a.normal_()
            g.eo_apply(a, b, m, prec, True, nrhs)  # first call: the odd inverse blocks
            torch.cuda.synchronize()
            reps = 20
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                g.eo_apply(a, b, m, prec, True, nrhs)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            gbs = eo_algorithmic_bytes(prec, nsites2, nrhs) / (ms * 1e-3) / 1e9
            out["eo_apply"][f"{name}_{nrhs}"] = {"ms": ms, "algorithmic_GB_s": gbs, "frac_of_8TB_s": gbs / 8000}
            log(f"[reweight] eo apply {name} nrhs {nrhs}: {ms:.3f} ms, {gbs:.0f} GB/s ({100 * gbs / 8000:.1f} %)")
            del a, b
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lw = g.log_w_eo(m, m + 0.01)
    out["log_w_eo"] = {"m_prime": m + 0.01, "value": lw, "s": time.perf_counter() - t0}
    log(f"[reweight] log W_eo(m, m+0.01) = {lw:.6e} in {out['log_w_eo']['s']:.3f} s")
    A, nu2, mu2, delta = cstar.ratapprox_quartic(8, 1e-2, 400.0)
    eta = g.new_native(1, cstar.FP64)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    eta.normal_(generator=gen)
    eta = eta[: eta.numel() // 2].contiguous().mul_(1 / np.sqrt(2.0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lwm, expo, st = g.w_mass(m, m + 0.01, nu2, mu2, eta, tol=1e-10)
    dt = time.perf_counter() - t0
    out["w_mass"] = {"n": 8, "range": [1e-2, 400.0], "delta": delta, "nsrc": 1, "tol": 1e-10, "log_w_mass": lwm,
                     "s": dt, "cg_iterations": st.cg_iterations, "eo_applies": st.eo_applies,
                     "ms_per_eo_apply": 1e3 * dt / max(1, st.eo_applies)}
    log(f"[reweight] W_mass: log {lwm:.6e}, {dt:.2f} s, {st.cg_iterations} CG iterations, {st.eo_applies} "
        f"even-odd applies, FP32 and FP64 rows ({out['w_mass']['ms_per_eo_apply']:.3f} ms each, all included)")
    g.close()
    del eta
    lb_args = argparse.Namespace(**vars(args))
    lb_args.lbar_tol = 1e-3
    out["lambda_bar"] = compare_lambda_bar(lb_args, su3_d, th_d, q, path[:1])
    fields = [synth.make_field(16, 16, w["eps"], 3000 + i, smear_steps=w["smear"], smear_backend="torch")
              for i in range(2)]
    t0 = time.perf_counter()
    st_e, signs, prods, secs = cstar.sign_ensemble(fields, [2 / 3, -1 / 3], [m, m], 16, 16, k=args.k,
                                                   eig=cstar.eig_opts(tol=args.tol, max_iter=1000))
    out["ensemble"] = {"lattice": "16x16^3", "seeds": [3000, 3001], "charges": [2 / 3, -1 / 3], "m_target": m,
                       "status": int(st_e), "signs": signs.tolist(), "products": prods.tolist(),
                       "seconds": secs.tolist(), "s": time.perf_counter() - t0}
    log(f"[reweight] ensemble 2 x 2 at 16^4: signs {signs.tolist()}, {out['ensemble']['s']:.1f} s")
    return out


def ensemble_probe(args, w):
    """cstar_sign_ensemble over n fields of the workload's distribution and
    size (drawn with the torch exponentials, host arrays handed to the
    driver), two flavours, sign at the lightest path mass: signs, flavour
    products and seconds per configuration."""
    import numpy as np

    from paper_2108_11989_amd import cstar, synth
    T, L = w["T"], w["L"]
    m = float(np.asarray(synth.kappa_to_m0(w["kappas"]), dtype=np.float64)[0])
    t0 = time.perf_counter()
    fields = [synth.make_field(T, L, w["eps"], 3000 + i, smear_steps=w["smear"], smear_backend="torch",
                               exp_backend="torch") for i in range(args.ensemble_probe)]
    t_fields = time.perf_counter() - t0
    t0 = time.perf_counter()
    st, signs, prods, secs = cstar.sign_ensemble(fields, [2 / 3, -1 / 3], [m, m], T, L, k=args.k,
                                                 eig=cstar.eig_opts(tol=args.tol, max_iter=1000))
    dt = time.perf_counter() - t0
    out = {"workload": args.workload, "lattice": f"{T}x{L}^3", "configurations": args.ensemble_probe,
           "seeds": [3000, 3000 + args.ensemble_probe - 1], "charges": [2 / 3, -1 / 3], "m_target": m,
           "k": args.k, "tol": args.tol, "status": int(st), "signs": signs.tolist(), "products": prods.tolist(),
           "seconds_per_configuration": secs.tolist(), "s": dt, "s_fields": t_fields,
           "signs_per_hour": 3600.0 * signs.size / dt}
    log(f"[ensemble] {args.ensemble_probe} configurations x 2 flavours at {T}x{L}^3: {dt:.1f} s, products "
        f"{prods.tolist()}, {out['signs_per_hour']:.0f} signs per hour")
    print(json.dumps({"ensemble_probe": out}), flush=True)


def c3(args, w):
    """The learned preconditioner at the workload's own size: trained on many
    fields of its distribution (streamed: a field, its plain-solver low modes,
    a few Adam steps, the next field), then judged on held-out fields against
    the plain solver (same filter, same tolerance)."""
    import numpy as np
    import torch

    from paper_2108_11989_amd import cstar, learned, synth
    T, L, q = w["T"], w["L"], w["q"][0]
    path = np.asarray(synth.kappa_to_m0(w["kappas"]), dtype=np.float64)
    m_train = float(path[0])

    def field(seed):
        su3, th = synth.make_field(T, L, w["eps"], seed, smear_steps=w["smear"], smear_backend="torch",
                                   exp_backend="torch")
        return cstar.Gauge(torch.from_numpy(su3).cuda(), torch.from_numpy(th).cuda(), q, synth.CSW_SU3,
                           synth.CSW_U1)

    out = {"workload": args.workload, "lattice": f"{T}x{L}^3", "q": q, "m0": m_train}
    if args.c3_train:
        t0 = time.perf_counter()
        net = cstar.Net(learned.initial_weights(m_train))

        def progress(i, h):
            np.save(args.c3_train, net.weights().astype(np.float32))  # a checkpoint after every field
            log(f"[c3] field {i}: loss {h[0]:.4f} -> {h[-1]:.4f} ({time.perf_counter() - t0:.0f} s)")

        hist = learned.train_online(net, lambda i: field(1000 + i), args.c3_fields, m_train, args.c3_steps, 1e-3,
                                    seed=7000, log=progress)
        np.save(args.c3_train, net.weights().astype(np.float32))
        net.close()
        out["train"] = {"fields": args.c3_fields, "seeds": [1000, 1000 + args.c3_fields - 1],
                        "pairs_per_field": 8, "low_modes_per_field": 4, "adam_steps_per_field": args.c3_steps,
                        "lr": 1e-3, "loss_first_field": [float(x) for x in hist[0]],
                        "loss_last_field": [float(x) for x in hist[-1]],
                        "loss_mean_first_8": float(hist[:8].mean()), "loss_mean_last_8": float(hist[-8:].mean()),
                        "s": time.perf_counter() - t0, "weights": args.c3_train}
        print(json.dumps({"c3_train": out}), flush=True)
        return
    wts = np.load(args.c3_eval, allow_pickle=False)
    net = cstar.Net(wts.astype(np.float32))
    solves = []
    for i in range(args.c3_test):
        g = field(2000 + i)
        row = {"seed": 2000 + i}
        for name, nn in (("plain_mixed", 0), ("learned_mixed", 1)):
            if nn:
                net.attach(g)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ev, res_, st = g.lowest_eigs(m_train, args.k, cstar.eig_opts(inner=cstar.FP32_BF16LINKS, tol=args.tol,
                                                                         max_iter=1000, use_nn=nn))
            row[name] = {"s": time.perf_counter() - t1, "iterations": st.iterations,
                         "applies": st.applies_inner + st.applies_fp64, "nn_applies": st.nn_applies,
                         "fallback": st.nn_fallback, "lambda": [float(x) for x in ev],
                         "resid_max": float(np.max(res_))}
            if nn:
                cstar.Net.detach(g)
        a, b = row["plain_mixed"], row["learned_mixed"]
        row["eigenvalues_agree"] = all(abs(x - y) <= a["resid_max"] + b["resid_max"] + 1e-12
                                       for x, y in zip(a["lambda"], b["lambda"]))
        log(f"[c3] test field {2000 + i}: plain {a['s']:.1f} s / {a['applies']} applies, learned {b['s']:.1f} s / "
            f"{b['applies']} applies + {b['nn_applies']} network, agree {row['eigenvalues_agree']}")
        solves.append(row)
        if i == 0 and args.c3_sign:
            out["sign"] = {}
            for name, nn in (("plain_mixed", 0), ("learned_mixed", 1)):
                g2 = field(2000)
                if nn:
                    net.attach(g2)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                sg, rep = g2.pfaffian_sign(path, k=args.k, eig=cstar.eig_opts(inner=cstar.FP32_BF16LINKS,
                                                                               tol=args.tol, max_iter=1000,
                                                                               use_nn=nn))
                out["sign"][name] = {"s": time.perf_counter() - t1, "applies": rep.applies,
                                     "nn_applies": rep.nn_applies, "points_solved": rep.n_points,
                                     "signs": "".join("+" if v > 0 else "-" for v in sg)}
                if nn:
                    cstar.Net.detach(g2)
                g2.close()
                log(f"[c3] sign {name}: {out['sign'][name]['s']:.1f} s, {out['sign'][name]['signs']}")
            out["sign"]["agree"] = out["sign"]["plain_mixed"]["signs"] == out["sign"]["learned_mixed"]["signs"]
        g.close()
    net.close()
    tot = {n: {"s": sum(r[n]["s"] for r in solves), "applies": sum(r[n]["applies"] for r in solves)}
           for n in ("plain_mixed", "learned_mixed")}
    out.update({"weights": args.c3_eval, "k": args.k, "tol": args.tol, "solves": solves, "totals": tot,
                "all_agree": all(r["eigenvalues_agree"] for r in solves)})
    print(json.dumps({"c3_eval": out}), flush=True)


def sign_path(args, w, su3_d, th_d, path, nsites2):
    """Pfaffian signs over the path for every charge of the workload, timed
    (profiling and paper-scale runs)."""
    import numpy as np
    import torch

    from paper_2108_11989_amd import cstar, synth
    inner = {"bf16": cstar.FP32_BF16LINKS, "fp32": cstar.FP32, "fp64": cstar.FP64}[args.inner]
    charges = [float(x) for x in w["q"]]
    if args.charges:
        charges = [charges[int(i)] for i in args.charges.split(",")]
    net = None
    opts = cstar.eig_opts(inner=inner, tol=args.tol, max_iter=1000, block=args.block)
    if args.learned:
        net, _ = train_network(args, w, charges[0], float(path[0]))
        opts = cstar.eig_opts(inner=inner, tol=args.tol, max_iter=1000, use_nn=1, block=args.block)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for qc in charges:
        g = cstar.Gauge(su3_d, th_d, qc, synth.CSW_SU3, synth.CSW_U1)
        if net is not None:
            net.attach(g)
        g.timing(True)
        tq = time.perf_counter()
        sg, rep = g.pfaffian_sign(path, k=args.k, eig=opts)
        tm = g.read_timing()
        g.close()
        res.append({"q": qc, "s": time.perf_counter() - tq, "mass_points_solved": rep.n_points,
                    "applies": rep.applies, "crossings": rep.n_crossings,
                    "signs": "".join("+" if v > 0 else "-" for v in sg), "timing": tm})
        log(f"[bench] q = {qc:+.4f}: {res[-1]['s']:.1f} s, {rep.n_points} points, {rep.applies} applies, "
            f"signs {res[-1]['signs']}")
    dt = time.perf_counter() - t0
    ms = [sum(r["timing"][p]["ms"] for r in res) for p in range(3)]
    dom = int(np.argmax(ms))
    launches = sum(r["timing"][dom]["launches"] for r in res)
    rhs = sum(r["timing"][dom]["rhs"] for r in res)
    operands = sum(r["timing"][dom]["operands"] for r in res)
    byts = algorithmic_bytes(dom, nsites2, launches, rhs, operands)
    achieved = byts / (ms[dom] * 1e-3) / 1e9 if ms[dom] > 0 else 0.0
    for r in res:
        del r["timing"]
    print(json.dumps({"sign_path": res, "workload": args.workload, "inner": args.inner, "learned": args.learned,
                      "s_total": dt, "applies_per_s": sum(r["applies"] for r in res) / dt,
                      "dominant_kernel": {"prec": dom, "launches": launches, "rhs_per_launch": rhs / max(launches, 1),
                                          "avg_ms": ms[dom] / max(launches, 1), "GBs": achieved,
                                          "frac": achieved / HBM_PEAK_GBS}}), flush=True)


if __name__ == "__main__":
    main()
