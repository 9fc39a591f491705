"""Benchmark of the HDCR hot path on one MI355X.

Workload: the 24^4 x 16 domain wall system (M5 = 1.8, mf = 0.01, periodic
boundaries with antiperiodic time, SU(3) links exp(0.3 i A) with A Gaussian
su(3), seed 1; complex Gaussian source, seed 0).

One timed step = one pass of the whole solve path on that system:
  * fine-operator sweep: 20 applications of H = Gamma5 D_dwf in FP64 and 20 in
    FP32 (rotating input/output buffers), each launch bracketed by HIP events on
    the stream it runs on;
  * the plain conjugate-residual solve to |b - Hx| <= 1e-8 |b| (FP64).
The printed value is the achieved algorithmic bandwidth of the FP64 fine
apply (bytes = 2 * 12 * N5 complex spinor entries + 36 * V4 link entries,
i.e. read psi once, write once, links once), averaged over the timed steps.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, nargs=4, default=[24, 24, 24, 24])
    ap.add_argument("--Ls", type=int, default=16)
    ap.add_argument("--applies", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-applies", type=int, default=8)
    return ap.parse_args()


def fine_bytes(V4, Ls, csize):
    return (2 * 12 * V4 * Ls + 36 * V4) * csize


def cpu_baseline(U, b, L, Ls, n_applies):
    """The FP64 oracle's fine apply on the host cores (a bounded sample: n_applies applications)."""
    import oracle
    p = oracle.Params(tuple(L), Ls, M5=1.8, mf=0.01)
    oracle.apply_h(U, b, p)  # warm up / load
    t0 = time.perf_counter()
    for _ in range(n_applies):
        oracle.apply_h(U, b, p)
    dt = (time.perf_counter() - t0) / n_applies
    V4 = int(np.prod(L))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(fine_bytes(V4, Ls, 16) / dt / 1e9, 3), "unit": "GB/s", "cores": cores,
            "kind": "oracle", "sample": f"{n_applies} FP64 applications of H at {'x'.join(map(str, L))}x{Ls} "
                                        f"({dt * 1e3:.0f} ms each)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path runs on one device)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import hdcr_inputs as hi
    import paper_1611_06944_amd as hd

    L, Ls = tuple(args.L), args.Ls
    lat = hd.Lattice(L, Ls, M5=1.8, mf=0.01)
    V4 = lat.V4
    U_aos = hi.gauge_field(L, seed=1)
    b_aos = hi.gaussian_fermion(L, Ls, seed=0)
    plaq = hi.plaquette(U_aos)
    dev = torch.device("cuda:0")
    U64 = torch.from_numpy(hd.pack_gauge(U_aos)).to(dev)
    b64 = torch.from_numpy(hd.pack_fermion(b_aos)).to(dev)
    U32 = U64.to(torch.complex64)
    base = {"c128": (U64, [b64.clone() for _ in range(2)], [torch.empty_like(b64) for _ in range(2)]),
            "c64": (U32, [b64.to(torch.complex64) for _ in range(2)],
                    [torch.empty(b64.shape, dtype=torch.complex64, device=dev) for _ in range(2)])}
    params = hd.default_params(tol=1e-8, maxiter=20000)
    work = torch.empty(hd.workspace_bytes(hd._abi.WS_SOLVE, lat, params), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def fine_sweep(prec, n):
        U, ins, outs = base[prec]
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for i in range(n):
            evs[i][0].record(stream)
            hd.apply_fine(lat, U, ins[i % 2], outs[i % 2])
            evs[i][1].record(stream)
        return evs

    def step():
        res = {}
        res["ev64"] = fine_sweep("c128", args.applies)
        res["ev32"] = fine_sweep("c64", args.applies)
        x = torch.zeros_like(b64)
        _, st, _ = hd.solve(lat, U64, b64, x, params=params, work=work)
        res["cr"] = st
        return res

    progress("inputs on device; warming up")
    for _ in range(args.warmup):
        r = step()
        progress(f"warmup step done (CR iters {r['cr']['outer_iters']}, {r['cr']['seconds_total']:.2f} s)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(step())
        progress(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    def avg_ms(key):
        return float(np.mean([a.elapsed_time(b) for r in results for a, b in r[key]]))

    ms64, ms32 = avg_ms("ev64"), avg_ms("ev32")
    gbs64 = fine_bytes(V4, Ls, 16) / (ms64 * 1e-3) / 1e9
    gbs32 = fine_bytes(V4, Ls, 8) / (ms32 * 1e-3) / 1e9
    cr = results[-1]["cr"]
    out = {
        "metric": "fine Γ5·D_dwf GB/s (% HBM peak); HDCR vs plain CR time-to-1e-8 at 24^4×16",
        "value": round(gbs64, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128 (fine apply value); c128 CR",
        "data": "synthetic (seeded SU(3) links exp(0.3iA), Gaussian source)",
        "config": {"workload": f"fine H apply + plain CR solve to 1e-8, {'x'.join(map(str, L))}x{Ls}, "
                               f"M5=1.8, mf=0.01, bc=(+,+,+,-)", "L": list(L), "Ls": Ls, "plaquette": round(plaq, 6)},
        "fine_apply": {"c128_us": round(ms64 * 1e3, 1), "c128_GBps": round(gbs64, 1),
                       "c128_pct_hbm": round(100 * gbs64 / HBM_PEAK_GBS, 1),
                       "c64_us": round(ms32 * 1e3, 1), "c64_GBps": round(gbs32, 1),
                       "c64_pct_hbm": round(100 * gbs32 / HBM_PEAK_GBS, 1),
                       "c128_GFLOPs": round(1416 * lat.N5 / (ms64 * 1e-3) / 1e9, 1),
                       "c64_GFLOPs": round(1416 * lat.N5 / (ms32 * 1e-3) / 1e9, 1)},
        "plain_cr": {"status": cr["status"], "iters": cr["outer_iters"], "seconds": round(cr["seconds_total"], 4),
                     "true_rel_residual": cr["true_rel_residual"], "fine_applies": cr["fine_applies_f64"]},
        "roofline": {"bound": "hbm", "achieved": round(gbs64, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs64 / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "dslash_dwf_kernel<double>", "bytes_per_launch": fine_bytes(V4, Ls, 16)},
    }
    if not args.no_cpu_baseline:
        progress("timing the CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(U_aos, b_aos, L, Ls, args.cpu_sample_applies)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
