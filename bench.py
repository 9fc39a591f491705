"""Benchmark of the HDCR hot path on one MI355X.

Workload: the 24^4 x 16 domain wall system H x = b, H = Gamma5 D_dwf (M5 = 1.8,
mf = 0.01, periodic boundaries with antiperiodic time; SU(3) links
exp(0.3 i A) with A Gaussian su(3), seed 1; complex Gaussian source, seed 0).

Setup (timed and reported on its own, as the paper reports its subspace
set-up apart from the solve): power iteration for lambda_max^2, 32 subspace
vectors by a degree-200 Chebyshev low-pass filter of seeded Gaussian noise
(FP32 arithmetic on FP16-stored fields), chirally split block basis on
4^4 x Ls blocks (Nb = 64, coarse 6^4) and the little Dirac operator in BF16
storage.

One timed step = one pass of the whole solve path on that system:
  * the HDCR solve to |b - Hx| <= 1e-8 |b| (FP64 flexible GCR(8), FP32
    two-level cycle with the order-10 Chebyshev smoother on [0.5, 64], the FP16
    copy of the basis for restriction and prolongation, coarse CR on the BF16
    little Dirac operator to 0.2);
  * the plain conjugate-residual solve of the same system (FP64);
  * a fine-operator sweep: 20 applications of H in FP32, 20 in FP64 and 20 with
    FP16 field storage, each launch bracketed by HIP events on the stream it
    runs on.
The printed value is the achieved algorithmic bandwidth of the FP32 fine apply
(the dominant kernel of the HDCR solve): bytes = (2 * 12 * N5 spinor entries +
36 * V4 link entries) * 8, i.e. psi read once, written once, links once.
Further sections: the project's copy-kernel ceiling, the deflated and
FP16-smoother solves, restriction, prolongation and the single-RHS coarse apply
at the solve's shape, the continued-fraction overlap operator, the batched
coarse apply on the matrix cores, the fermion force and the CPU oracle baseline.

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
    ap.add_argument("--block", type=int, nargs=4, default=[4, 4, 4, 4])
    ap.add_argument("--nvec", type=int, default=32)
    ap.add_argument("--degree", type=int, default=200, help="Chebyshev filter degree of the subspace set-up")
    ap.add_argument("--cut", type=float, default=0.02, help="filter cut lambda_cut^2 / lambda_max^2")
    ap.add_argument("--filter-storage", choices=["f32", "f16"], default="f16",
                    help="field storage of the subspace filter's recurrence (arithmetic FP32 either way)")
    ap.add_argument("--order", type=int, default=10, help="smoother terms (the paper: 10)")
    ap.add_argument("--cheb-lo", type=float, default=0.5,
                    help="smoother interval low end (the paper's ensemble: 1.0; tuned to the synthetic ensemble)")
    ap.add_argument("--cheb-hi", type=float, default=64.0)
    ap.add_argument("--basis", choices=["f32", "f16"], default="f16",
                    help="basis copy used by restriction/prolongation in the FP32 cycle")
    ap.add_argument("--coarse-tol", type=float, default=0.2)
    ap.add_argument("--restart", type=int, default=8)
    ap.add_argument("--applies", type=int, default=20)
    ap.add_argument("--fine-only", action="store_true", help="only the fine-operator sweep (for counter runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--force-only", action="store_true", help="only the fermion-force measurement (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 1 GiB device-to-device copies (reference for the HBM byte counters)")
    ap.add_argument("--cpu-sample-applies", type=int, default=6)
    ap.add_argument("--coarse-multi-only", action="store_true",
                    help="only the batched coarse apply sweep (profiling runs)")
    ap.add_argument("--cf-only", action="store_true", help="only the continued-fraction operator (profiling runs)")
    ap.add_argument("--basis-only", action="store_true",
                    help="only restriction, prolongation and the single-RHS coarse apply at the solve's shape, on "
                         "a constant-filled basis and a random A (profiling runs)")
    ap.add_argument("--defl-k", type=int, default=48, help="coarse deflation: eigenpairs kept (0: skip)")
    ap.add_argument("--defl-m", type=int, default=64, help="coarse deflation: block size of the set-up")
    ap.add_argument("--defl-degree", type=int, default=60)
    ap.add_argument("--defl-iters", type=int, default=5)
    ap.add_argument("--defl-only", action="store_true",
                    help="only the set-up and the deflated HDCR solve (profiling runs)")
    return ap.parse_args()


# HBM traffic of the FP32 fine apply at 24^4 x 16 from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by what they read for the library's copy kernel on 1 GiB), for
# the stencil sources (fine.hip and the shared header) with this sha256; reported as
# null for any other source or lattice.
MEASURED_TRAFFIC = {"stencil_sha256": "14924f7ffb113547d59de6a43e0e1cef575f9707de57c469d736d5aea6cc0030",
                    "L": [24, 24, 24, 24], "Ls": 16, "fp32_bytes_per_launch": 1862054912,
                    "summary": "profiles/dslash_fine_24x24x24x24x16_traffic.md"}


def stencil_sha256():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1611_06944_amd", "csrc")
    for f in ("fine.hip", "internal.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def measured_traffic(L, Ls):
    m = MEASURED_TRAFFIC
    if stencil_sha256() != m["stencil_sha256"] or list(L) != m["L"] or Ls != m["Ls"]:
        return None
    return m["fp32_bytes_per_launch"]


def fine_bytes(V4, Ls, csize):
    return (2 * 12 * V4 * Ls + 36 * V4) * csize


def cpu_model():
    """The host CPU's model name (lscpu's 'Model name', from /proc/cpuinfo) and its thread count."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name, os.cpu_count()


def cpu_baseline(U, b, L, Ls, n_applies, gpu_counts):
    """The FP64 oracle on the host cores, on bounded samples (about 20-30 s of CPU work).

    value: the oracle's fine apply at the benchmark lattice in algorithmic GB/s (n_applies
    applications).  legs: the other steps of the path measured directly where they fit the
    budget (coarse apply at the cfg-2 and cfg-3 coarse shapes), or timed on a smaller piece and
    scaled by the work ratio, labelled 'extrapolated': the coarse build (block basis and A per
    column, timed at 8^4 x 16 with the benchmark's blocks and Nb = 64, scaled by N5 and by the
    number of columns), plain CR and HDCR at 24^4 x 16 (the measured per-operation times times
    the operation counts of the GPU solves of the same system)."""
    import oracle
    import hdcr_inputs as hi
    p = oracle.Params(tuple(L), Ls, M5=1.8, mf=0.01)
    oracle.apply_h(U, b, p)  # warm up / load
    t0 = time.perf_counter()
    for _ in range(n_applies):
        oracle.apply_h(U, b, p)
    t_apply = (time.perf_counter() - t0) / n_applies
    V4 = int(np.prod(L))
    N5 = V4 * Ls
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model, threads = cpu_model()
    legs = {"fine_apply_s": round(t_apply, 4)}
    # numpy vector work of one CR iteration on fields of this size (2 inner products, 4 axpys, 1 norm)
    x, y = b.copy(), b.copy()
    t0 = time.perf_counter()
    for _ in range(2):
        a = np.vdot(x, y)
        x += 0.1 * y
        y -= 0.1 * x
        np.vdot(y, y)
        a = np.vdot(x, y)
        x += 0.1 * y
        y += 0.1 * x
    t_vec = (time.perf_counter() - t0) / 2
    del x, y
    legs["cr_vector_work_per_iter_s"] = round(t_vec, 4)
    # coarse apply at the cfg-2 (4^4, Nb 48) and cfg-3 (6^4, Nb 64) coarse shapes, Gaussian A
    rng = np.random.default_rng(5)
    t_capply = {}
    for name, cd, nb in (("cfg2_4x4x4x4_nb48", (4, 4, 4, 4), 48), ("cfg3_6x6x6x6_nb64", (6, 6, 6, 6), 64)):
        nc = int(np.prod(cd))
        A = rng.standard_normal((nc, 9, nb, nb)) + 1j * rng.standard_normal((nc, 9, nb, nb))
        v = rng.standard_normal((nc, nb)) + 1j * rng.standard_normal((nc, nb))
        oracle.coarse_apply(A, v, cd)
        t0 = time.perf_counter()
        for _ in range(5):
            oracle.coarse_apply(A, v, cd)
        t_capply[name] = (time.perf_counter() - t0) / 5
        legs[f"coarse_apply_{name}_s"] = round(t_capply[name], 5)
        del A
    # coarse build pieces at 8^4 x 16 with 4^4 blocks and nvec = 32 (Nb = 64)
    Ls_ = Ls
    Lb = (8, 8, 8, 8)
    pb = oracle.Params(Lb, Ls_, M5=1.8, mf=0.01)
    csb = oracle.Coarse(pb, (4, 4, 4, 4), 32)
    Ub = hi.gauge_field(Lb, seed=1)
    vecs = [hi.gaussian_fermion(Lb, Ls_, seed=100 + k) for k in range(32)]
    t0 = time.perf_counter()
    basis, _ = oracle.block_basis(vecs, csb)
    t_basis = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.coarse_columns(Ub, basis, csb, [0, 40])
    t_col = (time.perf_counter() - t0) / 2
    psi_b = vecs[0]
    t0 = time.perf_counter()
    oracle.prolong(basis, oracle.restrict(basis, psi_b, csb), csb)
    t_rp = time.perf_counter() - t0
    del vecs, basis
    N5b = int(np.prod(Lb)) * Ls_
    for name, n5, nvec in (("cfg2_16x16x16x16x16_nb48", 16 ** 4 * 16, 24), ("cfg3_24x24x24x24x16_nb64", 24 ** 4 * 16, 32)):
        r = n5 / N5b
        legs[f"coarse_build_{name}_s_extrapolated"] = round(t_basis * r * (nvec / 32) ** 2 + t_col * r * 2 * nvec, 1)
    tag = f"{'x'.join(map(str, L))}x{Ls}"
    t_rp24 = t_rp * N5 / N5b
    legs[f"restrict_plus_prolong_{tag}_nb64_s_extrapolated"] = round(t_rp24, 3)
    if gpu_counts:
        cr_it = gpu_counts["cr_iters"]
        legs[f"plain_cr_{tag}_s_extrapolated"] = round(cr_it * (t_apply + t_vec) + 2 * t_apply, 1)
        h = gpu_counts["hdcr"]
        # every fine apply at FP64 oracle cost, every coarse apply at the cfg-3 cost, one restriction
        # and prolongation per cycle (two cycles of smoothing share one coarse solve), FGCR vector
        # work of about one CR iteration's per outer iteration and window vector
        n_fine = h["fine_applies_inner"] + h["fine_applies_f64"]
        t_h = (n_fine * t_apply + h["coarse_applies"] * t_capply["cfg3_6x6x6x6_nb64"]
               + h["outer_iters"] * (t_rp24 + 8 * t_vec))
        legs[f"hdcr_{tag}_s_extrapolated"] = round(t_h, 1)
        legs["extrapolation_counts"] = {"cr_iters": cr_it, "hdcr_fine_applies": n_fine,
                                        "hdcr_coarse_applies": h["coarse_applies"], "hdcr_outer": h["outer_iters"]}
    return {"value": round(fine_bytes(V4, Ls, 16) / t_apply / 1e9, 3), "unit": "GB/s", "cores": cores,
            "kind": "oracle", "cpu_model": model, "host_threads": threads,
            "sample": f"{n_applies} FP64 applications of H at {'x'.join(map(str, L))}x{Ls} "
                      f"({t_apply * 1e3:.0f} ms each); legs as listed",
            "legs": legs}


def copy_ceiling(hd, torch):
    """The project's plain streaming copy kernel (hdcr_stream_copy) on 1 GiB: read + write bytes
    per second, the practical bandwidth ceiling beside the datasheet peak."""
    stream = torch.cuda.current_stream()
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        hd.stream_copy(src, dst)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
    for a_, b_ in evs:
        a_.record(stream)
        hd.stream_copy(src, dst)
        b_.record(stream)
    torch.cuda.synchronize()
    ms = float(np.median([a_.elapsed_time(b_) for a_, b_ in evs]))
    del src, dst
    torch.cuda.empty_cache()
    gbs = 2 * (1 << 30) / (ms * 1e-3) / 1e9
    return {"kernel": "hdcr_stream_copy, 1 GiB", "us": round(ms * 1e3, 1), "GBps": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def timed_launches(torch, fn, n=20):
    """Median ms of n launches of fn, each bracketed by HIP events on the current stream."""
    stream = torch.cuda.current_stream()
    for _ in range(3):
        fn()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a_, b_ in evs:
        a_.record(stream)
        fn()
        b_.record(stream)
    torch.cuda.synchronize()
    return float(np.median([a_.elapsed_time(b_) for a_, b_ in evs]))


def basis_section(hd, torch, lat, basis, A):
    """Restriction and prolongation of the two-level cycle (the whole basis streamed per call) and
    the single-RHS BF16 coarse apply of the coarse CR, at the solve's shape, each timed with HIP
    events over 20 launches: P^dag psi with the FP16 basis copy (the solve's choice) and with the
    FP32 one, P v with the FP16 copy, and A v.  Algorithmic bytes: the basis copy read once, psi
    read (restriction) or written (prolongation) once; A read once for the coarse apply."""
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(51)
    psi = torch.randn(lat.fshape, dtype=torch.complex64, device=dev, generator=gen)
    vc = torch.randn((lat.nc, lat.nb), dtype=torch.complex64, device=dev, generator=gen)
    outc = torch.empty_like(vc)
    outf = torch.empty_like(psi)
    f32 = 12 * lat.N5 * 8
    b16, b32 = lat.nvec * 12 * lat.N5 * 4, lat.nvec * 12 * lat.N5 * 8
    a_bytes = hd.coarse_bytes(lat, hd.BF16C)
    res = {"workload": f"{'x'.join(map(str, lat.L))}x{lat.Ls}, blocks {'x'.join(map(str, lat.block))}, "
                       f"Nb={lat.nb}, coarse {lat.nc} sites"}
    cases = (("restrict_f16_basis", lambda: hd.restrict(lat, basis, psi, out=outc, half_basis=True), b16 + f32),
             ("restrict_f32_basis", lambda: hd.restrict(lat, basis, psi, out=outc), b32 + f32),
             ("prolong_f16_basis", lambda: hd.prolong(lat, basis, vc, out=outf, half_basis=True), b16 + f32),
             ("coarse_apply_bf16", lambda: hd.apply_coarse(lat, A, hd.BF16C, vc, outc), a_bytes))
    for name, fn, nbytes in cases:
        ms = timed_launches(torch, fn)
        res[name] = {"us": round(ms * 1e3, 1), "bytes_per_launch": nbytes,
                     "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del psi, vc, outc, outf
    return res


def cf_section(hd, hi, torch):
    """The continued-fraction overlap operator (Sec. 3) at 24^4 with 8 pole slices (Ls = 9) and
    with 15 (Ls = 16): the seeded links, Gaussian field, beta_i spaced evenly in [0.5, 2], R = 0.3.
    Algorithmic bytes as for H: the field read and written once, the links once."""
    dev = torch.device("cuda:0")
    L = (24, 24, 24, 24)
    Uh = hd.pack_gauge(hi.gauge_field(L, seed=hi.LINK_SEED))
    gen = torch.Generator(device=dev)
    gen.manual_seed(41)
    res = {"workload": "24x24x24x24, M5=1.8, beta_i in [0.5, 2], R=0.3 (synthetic)"}
    for m in (8, 15):
        Ls = m + 1
        lat = hd.Lattice(L, Ls, M5=1.8)
        beta = list(np.linspace(0.5, 2.0, m))
        for name, dt, cb in (("c64", torch.complex64, 8), ("c128", torch.complex128, 16)):
            U = torch.from_numpy(Uh).to(dev).to(dt)
            x = torch.randn((12, lat.V4, Ls), dtype=dt, device=dev, generator=gen)
            o = torch.empty_like(x)
            ms = timed_launches(torch, lambda: hd.apply_cf(lat, U, x, beta, 0.3, out=o))
            nbytes = fine_bytes(lat.V4, Ls, cb)
            res[f"Ls{Ls}_{name}"] = {"us": round(ms * 1e3, 1), "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
                                     "frac_hbm": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                     "bytes_per_launch": nbytes}
            del U, x, o
    torch.cuda.empty_cache()
    return res


def coarse_multi_section(hd, torch):
    """Multi-RHS coarse apply (16^4 x 16 fine, coarse 4^4 from 4^4 blocks, Nb = 64, BF16 A with
    Gaussian entries) on the matrix cores, at 12, 48, 96 and 192 right-hand sides: the autotuned
    tile shape with the vectors rounded to bf16, and the same apply with each complex64 entry
    carried as three bf16 terms (exact products, FP32 sums: the complex64 apply of the stored A).
    At 12 right-hand sides (the multi-RHS configuration) also one single-RHS launch per
    right-hand side and the complex64 vector-unit multi-RHS kernel on a C64 copy of A."""
    dev = torch.device("cuda:0")
    latc = hd.Lattice((16, 16, 16, 16), 16, block=(4, 4, 4, 4), nvec=32)
    gen = torch.Generator(device=dev)
    gen.manual_seed(21)
    raw = torch.randn(hd.coarse_bytes(latc, hd.C128) // 8, dtype=torch.float64, device=dev, generator=gen)
    Ab = hd.convert_coarse(latc, raw, hd.BF16C)
    A64 = hd.convert_coarse(latc, raw, hd.C64)
    del raw
    a_bytes = hd.coarse_bytes(latc, hd.BF16C)
    res = {"workload": "16x16x16x16x16, coarse 4^4, Nb=64, bf16 A (synthetic)"}
    for nrhs in (12, 48, 96, 192):
        v = torch.randn((nrhs, latc.nc, latc.nb), dtype=torch.complex64, device=dev, generator=gen)
        out = torch.empty_like(v)
        best, ms = hd.tune_coarse_batched(latc, Ab, v, out)
        t_b = timed_launches(torch, lambda: hd.apply_coarse_batched(latc, Ab, v, out))
        t_3 = timed_launches(torch, lambda: hd.apply_coarse_batched(latc, Ab, v, out, terms=3))
        flops = 8.0 * latc.nb * latc.nb * 9 * latc.nc * nrhs
        r = {"batched_variant": best, "variant_ms": [round(x, 4) for x in ms], "batched_us": round(t_b * 1e3, 1),
             "A_GBps": round(a_bytes / (t_b * 1e-3) / 1e9, 1),
             "mfma_TFLOPs": round(flops / (t_b * 1e-3) / 1e12, 2),
             "mfma_frac_bf16_peak": round(flops / (t_b * 1e-3) / 2.5e15, 5),
             "c64_exact_3terms_us": round(t_3 * 1e3, 1),
             "c64_exact_3terms_TFLOPs": round(flops / (t_3 * 1e-3) / 1e12, 2)}
        if nrhs == 12:
            t_1 = timed_launches(torch, lambda: [hd.apply_coarse(latc, Ab, hd.BF16C, v[q], out[q])
                                                 for q in range(nrhs)])
            t_c64 = timed_launches(torch, lambda: hd.apply_coarse(latc, A64, hd.C64, v, out))
            r.update({"single_rhs_loop_us": round(t_1 * 1e3, 1), "speedup_vs_loop": round(t_1 / t_b, 2),
                      "c64_valu_multi_rhs_us": round(t_c64 * 1e3, 1),
                      "c64_valu_TFLOPs": round(flops / (t_c64 * 1e-3) / 1e12, 2)})
        res[f"nrhs{nrhs}"] = r
        del v, out
    del Ab, A64
    torch.cuda.empty_cache()
    return res


def force_section(hd, hi, torch):
    """Fermion force of L = Re <chi, H psi> (16^4 x 16, Gaussian chi and psi): link gradient W and
    su(3) force T in one launch, FP64 and FP32.  'cold': a 512 MiB copy before every launch evicts
    L2 and the last-level cache, so the inputs come from HBM; 'warm': back-to-back launches (the
    FP32 inputs fit the 256 MB last-level cache).  Also the two launches of the autograd backward
    (H grad_y for psi, W for U)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    Lf, Lsf = (16, 16, 16, 16), 16
    latf = hd.Lattice(Lf, Lsf)
    Uf = hd.pack_gauge(hi.gauge_field(Lf, seed=hi.LINK_SEED))
    gen = torch.Generator(device=dev)
    gen.manual_seed(31)
    flush_a = torch.empty(1 << 29, dtype=torch.uint8, device=dev)
    flush_b = torch.empty_like(flush_a)
    res = {"workload": "16x16x16x16x16, Gaussian chi and psi, W and T per launch"}
    for name, dt, cb in (("c128", torch.complex128, 16), ("c64", torch.complex64, 8)):
        Ud = torch.from_numpy(Uf).to(dev).to(dt)
        chi = torch.randn((12, latf.V4, Lsf), dtype=dt, device=dev, generator=gen)
        psi = torch.randn((12, latf.V4, Lsf), dtype=dt, device=dev, generator=gen)
        W, T = torch.empty_like(Ud), torch.empty_like(Ud)
        Hg = torch.empty_like(chi)

        def launch():
            hd.fermion_force(latf, Ud, chi, psi, W, T)

        def per_launch(fn, n, flush):
            for _ in range(3):
                fn()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
            for a_, b_ in evs:
                if flush:
                    flush_b.copy_(flush_a)
                a_.record(stream)
                fn()
                b_.record(stream)
            torch.cuda.synchronize()
            return float(np.median([a_.elapsed_time(b_) for a_, b_ in evs]))

        cold = per_launch(launch, 20, True)
        warm = per_launch(launch, 20, False)
        bwd = per_launch(lambda: (hd.apply_fine(latf, Ud, chi, Hg),
                                  hd.fermion_force(latf, Ud, chi, psi, W, None, want_t=False)), 20, True)
        nbytes = latf.V4 * (24 * Lsf + 36 + 72) * cb
        res[name] = {"cold_us": round(cold * 1e3, 1), "warm_us": round(warm * 1e3, 1),
                     "cold_GBps": round(nbytes / (cold * 1e-3) / 1e9, 1),
                     "cold_pct_hbm": round(100 * nbytes / (cold * 1e-3) / 1e9 / HBM_PEAK_GBS, 1),
                     "warm_GBps": round(nbytes / (warm * 1e-3) / 1e9, 1),
                     "bytes_per_launch": nbytes, "backward_cold_us": round(bwd * 1e3, 1)}
        del Ud, chi, psi, W, T, Hg
    del flush_a, flush_b
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path runs on one device)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import hdcr_inputs as hi
    import paper_1611_06944_amd as hd

    if args.copy_calibration:
        # the project's copy kernel on 1 GiB, five times: the reference of the traffic counters
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            hd.stream_copy(src, dst)
        torch.cuda.synchronize()
        print("copied 5 x 1 GiB with hdcr_stream_copy", flush=True)
        return
    if args.force_only:
        print(json.dumps({"fermion_force": force_section(hd, hi, torch)}), flush=True)
        return
    if args.coarse_multi_only:
        print(json.dumps({"coarse_multi_rhs": coarse_multi_section(hd, torch)}), flush=True)
        return
    if args.cf_only:
        print(json.dumps({"cf_overlap": cf_section(hd, hi, torch)}), flush=True)
        return
    if args.basis_only:
        latb = hd.Lattice(tuple(args.L), args.Ls, M5=1.8, mf=0.01, block=tuple(args.block), nvec=args.nvec)
        bas = torch.full((hd.basis_bytes(latb),), 60, dtype=torch.uint8, device="cuda:0")  # 0x3c3c: small finite values
        gen = torch.Generator(device="cuda:0")
        gen.manual_seed(52)
        raw = torch.randn(hd.coarse_bytes(latb, hd.C128) // 8, dtype=torch.float64, device="cuda:0", generator=gen)
        Ab = hd.convert_coarse(latb, raw, hd.BF16C)
        del raw
        print(json.dumps({"basis_transfer": basis_section(hd, torch, latb, bas, Ab)}), flush=True)
        return

    L, Ls = tuple(args.L), args.Ls
    lat = hd.Lattice(L, Ls, M5=1.8, mf=0.01, block=tuple(args.block), nvec=args.nvec)
    V4 = lat.V4
    t_in = time.perf_counter()
    U_aos = hi.gauge_field(L, seed=1)
    b_aos = hi.gaussian_fermion(L, Ls, seed=0)
    plaq = hi.plaquette(U_aos)
    dev = torch.device("cuda:0")
    U64 = torch.from_numpy(hd.pack_gauge(U_aos)).to(dev)
    b64 = torch.from_numpy(hd.pack_fermion(b_aos)).to(dev)
    U32 = U64.to(torch.complex64)
    sweep = {"c128": (U64, [b64.clone() for _ in range(2)], [torch.empty_like(b64) for _ in range(2)]),
             "c64": (U32, [b64.to(torch.complex64) for _ in range(2)],
                     [torch.empty(b64.shape, dtype=torch.complex64, device=dev) for _ in range(2)]),
             # FP16 field storage (fp16 re, fp16 im), FP32 links
             "f16": (U32, [torch.view_as_real(b64.to(torch.complex64)).to(torch.float16).contiguous()
                           for _ in range(2)],
                     [torch.empty(b64.shape + (2,), dtype=torch.float16, device=dev) for _ in range(2)])}
    torch.cuda.synchronize()
    progress(f"inputs on device ({time.perf_counter() - t_in:.1f} s, plaquette {plaq:.6f})")
    stream = torch.cuda.current_stream()

    def fine_sweep(prec, n):
        U, ins, outs = sweep[prec]
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for i in range(n):
            evs[i][0].record(stream)
            hd.apply_fine(lat, U, ins[i % 2], outs[i % 2])
            evs[i][1].record(stream)
        return evs

    setup = {}
    if not args.fine_only:
        # ---- set-up: subspace and coarse space ----
        t0 = time.perf_counter()
        lam = hd.power_max(lat, U64, hi.gaussian_fermion_device(L, Ls, 99), iters=30)
        hi2 = 1.1 * lam
        vecs = torch.empty((args.nvec, 12, V4, Ls), dtype=torch.complex128, device=dev)
        sub_work = None
        for k in range(args.nvec):
            noise = hi.gaussian_fermion_device(L, Ls, hi.SUBSPACE_SEED0 + k).unsqueeze(0).contiguous()
            vecs[k:k + 1] = hd.make_subspace(lat, U64, noise, args.degree, args.cut * hi2, hi2,
                                             dtype=hd.F16C if args.filter_storage == "f16" else hd.C64, work=sub_work)
            del noise
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        basis, A = hd.build_coarse(lat, U64, vecs, hd.BF16C)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        del vecs
        torch.cuda.empty_cache()
        setup = {"solver": {"smoother_order": args.order, "smoother_interval": [args.cheb_lo, args.cheb_hi],
                            "coarse_tol": args.coarse_tol, "fgcr_restart": args.restart, "inner": "c64",
                            "coarse": "bf16c", "basis_restrict_prolong": args.basis},
                 "lambda_max_sq": round(lam, 4), "filter_degree": args.degree, "nvec": args.nvec,
                 "filter_storage": args.filter_storage,
                 "subspace_s": round(t1 - t0, 3), "coarse_build_s": round(t2 - t1, 3)}
        progress(f"set-up done: subspace {t1 - t0:.1f} s, coarse build {t2 - t1:.1f} s")
        prm_hdcr = hd.default_params(precond=hd.PRECOND_TWO_LEVEL, inner_dtype=hd.C64, coarse_dtype=hd.BF16C,
                                     coarse_tol=args.coarse_tol, coarse_maxiter=500, restart=args.restart, tol=1e-8,
                                     maxiter=500, cheb_order=args.order, cheb_lo=args.cheb_lo, cheb_hi=args.cheb_hi,
                                     basis_dtype=hd.F16C if args.basis == "f16" else hd.C64)
        prm_cr = hd.default_params(tol=1e-8, maxiter=20000)
        work_hdcr = torch.empty(hd.workspace_bytes(hd._abi.WS_SOLVE, lat, prm_hdcr), dtype=torch.uint8, device=dev)
        work_cr = torch.empty(hd.workspace_bytes(hd._abi.WS_SOLVE, lat, prm_cr), dtype=torch.uint8, device=dev)

    def step():
        res = {}
        if not args.fine_only:
            x = torch.zeros_like(b64)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, st, _ = hd.solve(lat, U64, b64, x, params=prm_hdcr, basis=basis, A=A, work=work_hdcr)
            res["hdcr"] = st
            res["hdcr_wall"] = time.perf_counter() - t
            x = torch.zeros_like(b64)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, st, _ = hd.solve(lat, U64, b64, x, params=prm_cr, work=work_cr)
            res["cr"] = st
            res["cr_wall"] = time.perf_counter() - t
        res["ev32"] = fine_sweep("c64", args.applies)
        res["ev64"] = fine_sweep("c128", args.applies)
        res["ev16"] = fine_sweep("f16", args.applies)
        return res

    defl_space = {}

    def f16_section():
        """The HDCR solve with the smoother's fields stored in FP16 (inner_dtype F16C; everything
        else as in hdcr_vs_cr), without and with the coarse deflation space."""
        prm = hd.default_params(precond=hd.PRECOND_TWO_LEVEL, inner_dtype=hd.F16C, coarse_dtype=hd.BF16C,
                                coarse_tol=args.coarse_tol, coarse_maxiter=500, restart=args.restart, tol=1e-8,
                                maxiter=500, cheb_order=args.order, cheb_lo=args.cheb_lo, cheb_hi=args.cheb_hi,
                                basis_dtype=hd.F16C if args.basis == "f16" else hd.C64)
        work = torch.empty(hd.workspace_bytes(hd._abi.WS_SOLVE, lat, prm), dtype=torch.uint8, device=dev)
        res = {}
        for name, d in (("no_deflation", None), ("deflation", defl_space.get("d"))):
            if name == "deflation" and d is None:
                continue
            runs = []
            for _ in range(max(1, args.steps)):
                x = torch.zeros_like(b64)
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, st, _ = hd.solve(lat, U64, b64, x, params=prm, basis=basis, A=A, work=work, defl=d)
                runs.append(time.perf_counter() - t)
            res[name] = {"solve_s": round(float(np.mean(runs)), 4), "outer_iters": st["outer_iters"],
                         "coarse_iters": st["coarse_iters"], "coarse_breakdowns": st["coarse_breakdowns"],
                         "fine_s": round(st["seconds_fine"], 4),
                         "coarse_s": round(st["seconds_coarse"], 4), "true_rel_residual": st["true_rel_residual"],
                         "status": st["status"]}
        return res

    def deflation_section():
        """Coarse-space eigenvector deflation: set-up time, then the HDCR solve of the timed
        steps with every coarse CR started from the Galerkin projection on the deflation space."""
        gen = torch.Generator(device=dev)
        gen.manual_seed(31)
        v0 = torch.randn((args.defl_m, lat.nc, lat.nb), dtype=torch.complex128, device=dev, generator=gen)
        hd.build_deflation(lat, A, hd.BF16C, v0, args.defl_k, degree=args.defl_degree, iters=args.defl_iters)
        torch.cuda.synchronize()
        t = time.perf_counter()
        d = hd.build_deflation(lat, A, hd.BF16C, v0, args.defl_k, degree=args.defl_degree, iters=args.defl_iters)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t
        del v0
        runs = []
        for _ in range(max(1, args.steps)):
            x = torch.zeros_like(b64)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, st, _ = hd.solve(lat, U64, b64, x, params=prm_hdcr, basis=basis, A=A, work=work_hdcr, defl=d)
            runs.append((time.perf_counter() - t, st))
        w = float(np.mean([r[0] for r in runs]))
        st = runs[-1][1]
        # eigenpair residuals |A v - theta v| (|v| = 1) of the stored operator
        res = (d.W - d.theta.to(d.V.real.dtype)[:, None, None] * d.V).reshape(d.k, -1).norm(dim=1)
        defl_space["d"] = d
        return {"k": args.defl_k, "k_found": d.k, "m": args.defl_m, "degree": args.defl_degree, "passes": args.defl_iters,
                "setup_s": round(t_setup, 3), "ritz_abs_min_max": [round(abs(d.theta_host[0]), 5),
                                                                  round(abs(d.theta_host[-1]), 5)],
                "ritz_residual_max": float(res.max()),
                "hdcr_defl_solve_s": round(w, 4), "outer_iters": st["outer_iters"],
                "coarse_iters": st["coarse_iters"], "coarse_breakdowns": st["coarse_breakdowns"],
                "coarse_s": round(st["seconds_coarse"], 4),
                "fine_s": round(st["seconds_fine"], 4), "outer_s": round(st["seconds_outer"], 4),
                "true_rel_residual": st["true_rel_residual"], "status": st["status"]}

    if args.defl_only:
        print(json.dumps({"coarse_deflation": deflation_section()}), flush=True)
        return

    for _ in range(args.warmup):
        r = step()
        if not args.fine_only:
            progress(f"warmup step done (HDCR {r['hdcr']['outer_iters']} it {r['hdcr_wall']:.2f} s, "
                     f"CR {r['cr']['outer_iters']} it {r['cr_wall']:.2f} s)")
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

    ms64, ms32, ms16 = avg_ms("ev64"), avg_ms("ev32"), avg_ms("ev16")
    bytes16 = 2 * 12 * V4 * Ls * 4 + 36 * V4 * 8   # FP16 fields, FP32 links
    gbs16 = bytes16 / (ms16 * 1e-3) / 1e9
    gbs64 = fine_bytes(V4, Ls, 16) / (ms64 * 1e-3) / 1e9
    gbs32 = fine_bytes(V4, Ls, 8) / (ms32 * 1e-3) / 1e9
    out = {
        "metric": "fine Γ5·D_dwf GB/s (% HBM peak); HDCR vs plain CR time-to-1e-8 at 24^4×16",
        "value": round(gbs32, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 fine apply (value); c128 outer FGCR / plain CR; bf16 coarse storage",
        "data": "synthetic (seeded SU(3) links exp(0.3iA), Gaussian source and subspace noise)",
        "config": {"workload": f"HDCR and plain CR to 1e-8 + fine H sweeps, {'x'.join(map(str, L))}x{Ls}, "
                               f"M5=1.8, mf=0.01, bc=(+,+,+,-), blocks {'x'.join(map(str, args.block))}xLs, "
                               f"Nb={2 * args.nvec}", "L": list(L), "Ls": Ls, "plaquette": round(plaq, 6)},
        "fine_apply": {"c64_us": round(ms32 * 1e3, 1), "c64_GBps": round(gbs32, 1),
                       "c64_pct_hbm": round(100 * gbs32 / HBM_PEAK_GBS, 1),
                       "c128_us": round(ms64 * 1e3, 1), "c128_GBps": round(gbs64, 1),
                       "c128_pct_hbm": round(100 * gbs64 / HBM_PEAK_GBS, 1),
                       "c64_GFLOPs": round(1416 * lat.N5 / (ms32 * 1e-3) / 1e9, 1),
                       "c128_GFLOPs": round(1416 * lat.N5 / (ms64 * 1e-3) / 1e9, 1),
                       "f16_storage_us": round(ms16 * 1e3, 1), "f16_storage_GBps": round(gbs16, 1),
                       "f16_storage_pct_hbm": round(100 * gbs16 / HBM_PEAK_GBS, 1),
                       "f16_storage_bytes_per_launch": bytes16},
        "roofline": {"bound": "hbm", "achieved": round(gbs32, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs32 / HBM_PEAK_GBS, 4), "traffic": measured_traffic(L, Ls), "traffic_unit": "B/launch",
                     "kernel": "dslash_par2_kernel<0>", "bytes_per_launch": fine_bytes(V4, Ls, 8)},
    }
    if not args.fine_only:
        h, c = results[-1]["hdcr"], results[-1]["cr"]
        hw = float(np.mean([r["hdcr_wall"] for r in results]))
        cw = float(np.mean([r["cr_wall"] for r in results]))
        out["hdcr_vs_cr"] = {
            "speedup": round(cw / hw, 3),
            "hdcr_solve_s": round(hw, 4), "cr_solve_s": round(cw, 4),
            "hdcr": {"outer_iters": h["outer_iters"], "coarse_iters": h["coarse_iters"],
                     "coarse_breakdowns": h["coarse_breakdowns"],
                     "fine_applies_f32": h["fine_applies_inner"], "fine_applies_f64": h["fine_applies_f64"],
                     "true_rel_residual": h["true_rel_residual"], "status": h["status"],
                     "fine_s": round(h["seconds_fine"], 4), "coarse_s": round(h["seconds_coarse"], 4),
                     "outer_s": round(h["seconds_outer"], 4)},
            "cr": {"iters": c["outer_iters"], "fine_applies_f64": c["fine_applies_f64"],
                   "true_rel_residual": c["true_rel_residual"], "status": c["status"]},
            "setup": setup,
            "setup_plus_solve_s": round(hw + setup.get("subspace_s", 0) + setup.get("coarse_build_s", 0), 3),
        }
    if not args.fine_only and args.defl_k > 0:
        dsec = deflation_section()
        dsec["speedup_vs_cr"] = round(cw / dsec["hdcr_defl_solve_s"], 3)
        dsec["speedup_vs_hdcr"] = round(hw / dsec["hdcr_defl_solve_s"], 3)
        out["coarse_deflation"] = dsec
        progress("deflated HDCR solve measured")
    if not args.fine_only:
        fsec = f16_section()
        for v in fsec.values():
            v["speedup_vs_cr"] = round(cw / v["solve_s"], 3)
        out["hdcr_f16_smoother"] = fsec
        progress("HDCR with the FP16-storage smoother measured")
    if not args.fine_only:
        out["basis_transfer"] = basis_section(hd, torch, lat, basis, A)
        progress("restriction, prolongation and single-RHS coarse apply measured")
        del basis, A, work_hdcr, work_cr
        defl_space.clear()
        torch.cuda.empty_cache()
        out["coarse_multi_rhs"] = coarse_multi_section(hd, torch)
        progress("multi-RHS coarse apply measured")
        out["cf_overlap"] = cf_section(hd, hi, torch)
        progress("continued-fraction operator measured")
        out["fermion_force"] = force_section(hd, hi, torch)
        progress("fermion force measured")
    out["copy_ceiling"] = copy_ceiling(hd, torch)
    out["roofline"]["copy_ceiling_GBps"] = out["copy_ceiling"]["GBps"]
    out["roofline"]["frac_of_copy_ceiling"] = round(gbs32 / out["copy_ceiling"]["GBps"], 4)
    if not args.no_cpu_baseline:
        progress("timing the CPU oracle baseline")
        counts = None
        if not args.fine_only:
            counts = {"cr_iters": c["outer_iters"], "hdcr": h}
        out["cpu_baseline"] = cpu_baseline(U_aos, b_aos, L, Ls, args.cpu_sample_applies, counts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
