"""Profiling helpers for the hot-path kernels.

    python -m paper_2112_02211_amd.profile_run [run] [--workload NAME] [--launches 4] [--lambda-bucket D]
    python -m paper_2112_02211_amd.profile_run pmc-summary --fetch DIR --write DIR --out FILE
    python -m paper_2112_02211_amd.profile_run arnoldi [--workload NAME]
    python -m paper_2112_02211_amd.profile_run arnoldi-summary --fetch DIR --write DIR --run-log FILE --out FILE
    python -m paper_2112_02211_amd.profile_run gemm [--workload NAME] [--rhs 64]
    python -m paper_2112_02211_amd.profile_run gemm-summary --pmc-dir DIR --out FILE
    python -m paper_2112_02211_amd.profile_run trace-summary --stats CSV --out FILE --cmd CMD --title T

``run`` (the default) is the fixed launch sequence for hardware-counter runs:
it sets up the workload (FP64, FP32 and BF16 blocks), then launches, each
--launches times after one warm-up: the operator apply (sweep + exchange),
the left-preconditioned operator J^{-1} A (sweep, then J^{-1} with the face
exchange fused into its load: the variant the solver runs and the benchmark's
roofline times), the preconditioner alone in each block precision, and a
plain elementwise kernel over --copy-mib MiB (dst = 2 src: each byte read once
and written once; the known-size reference that calibrates the FETCH_SIZE /
WRITE_SIZE counters).  Prints one line per phase with its wall time.

``pmc-summary`` turns two rocprofv3 --pmc runs of ``run`` (one FETCH_SIZE, one
WRITE_SIZE, csv output) into the traffic summary that bench.py reads.
``arnoldi`` solves the workload twice with the separable J^-1 (the second
solve with every Arnoldi update pass event-timed, printing their number and
algorithmic bytes), then runs the calibration kernel; ``arnoldi-summary``
turns its two counter runs into the update pass's traffic summary.
``gemm`` launches J^{-1} on --rhs right-hand sides (the block product as a
GEMM on the matrix cores) with FP64, FP32 and BF16 blocks; ``gemm-summary``
turns one counter run of it (MfmaUtil and the MFMA operation counts) into the
matrix-core summary of the block GEMM.
``trace-summary`` turns a rocprofv3 --kernel-trace --stats kernel_stats.csv
into a text table.
"""
import argparse
import collections
import csv
import hashlib
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CSRC = os.path.join(ROOT, "paper_2112_02211_amd", "csrc")
# every source the preconditioner kernel is compiled from
PRECOND_SOURCES = ("k_precond_fused.h", "k_leaf.h", "k_common.h")
# the Arnoldi kernels and their launchers
ARNOLDI_SOURCES = ("k_dcgs.hip", "k_common.h", "k_vec.h")
KERNEL_SOURCES = {"k_precond_fused": PRECOND_SOURCES, "k_dcgs_update": ARNOLDI_SOURCES}
COPY_MIB = 1024


def kernel_source_hash(kernel: str = "k_precond_fused") -> str:
    """Hash of a profiled kernel's sources: counters taken on other sources
    describe another kernel."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def run(a):
    import numpy as np
    import torch
    from paper_2112_02211_amd import hps, problems as P

    prob = P.workload(a.workload)
    ctx = hps.Context.from_problem(prob, block_precs=("fp64", "fp32", "bf16"),
                                   lambda_bucket=a.lambda_bucket)
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.standard_normal(ctx.N) + 1j * rng.standard_normal(ctx.N)).cuda()
    y = torch.empty_like(x)
    phases = [("apply", lambda: ctx.apply(x, y)), ("op_left", lambda: ctx.op_left(x, y))] + \
             [(f"precond_{q}", (lambda q=q: ctx.precond(x, y, prec=q))) for q in ("fp64", "fp32", "bf16")]
    if a.iti:
        # the face-reduced operator (exact ItI maps): its block product and exchange
        ctx.iti_build()
        f = torch.from_numpy(rng.standard_normal(ctx.nl * ctx.nb) + 0j).cuda()
        g = torch.empty_like(f)
        phases.append(("iti_apply", lambda: ctx.iti_apply(f, g)))
    n = a.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    phases.append(("copy", lambda: torch.mul(src, 2.0, out=dst)))
    for name, fn in phases:
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.launches):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.launches
        print(f"{name}: {dt * 1e3:.4f} ms per launch", flush=True)
    print(f"copy bytes read = written = {n * 4}")


def sep(a):
    """The kernels of one step of the separable solve, --launches times each
    after one warm-up: the left operator J^-1 A (sweep, then the separable J^-1
    with the exchange fused into its load) on complex FP64 vectors and on
    complex FP32 vectors (the inner step of iterative refinement)."""
    import numpy as np
    import torch
    from paper_2112_02211_amd import hps, problems as P

    prob = P.workload(a.workload)
    ctx = hps.Context.from_problem(prob, block_precs=("separable",))
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.standard_normal(ctx.N) + 1j * rng.standard_normal(ctx.N)).cuda()
    y = torch.empty_like(x)
    x32 = x.to(torch.complex64)
    y32 = torch.empty_like(x32)
    for name, fn in (("op_left_fp64", lambda: ctx.op_left(x, y)),
                     ("op_left_fp32", lambda: ctx.op_left_f32(x32, y32))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.launches):
            fn()
        torch.cuda.synchronize()
        print(f"{name}: {(time.perf_counter() - t0) / a.launches * 1e3:.4f} ms per launch", flush=True)


SQ_DOC = {
    "SQ_WAVES": "waves launched",
    "SQ_WAVE_CYCLES": "wave-cycles resident (summed over waves)",
    "SQ_BUSY_CYCLES": "cycles the sequencers were busy",
    "SQ_INSTS_VALU": "vector ALU instructions",
    "SQ_ACTIVE_INST_VALU": "cycles a wave issued VALU work (summed over waves)",
    "SQ_INSTS_LDS": "LDS instructions",
    "SQ_LDS_BANK_CONFLICT": "cycles stalled on LDS bank conflicts",
    "SQ_INSTS_VMEM_RD": "vector memory read instructions",
    "GRBM_GUI_ACTIVE": "GPU busy cycles",
}


def sq_summary(a):
    """Per-kernel sequencer counters (one --pmc run, csv in --pmc-dir) of the
    kernels whose names contain the --kernels substrings: averages per
    dispatch, and the derived occupancy (resident waves per CU), VALU-active
    and LDS-conflict fractions."""
    path = os.path.join(a.pmc_dir, "run_counter_collection.csv")
    rows = list(csv.DictReader(open(path)))
    by = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        by[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    L = [f"# {a.title}", "#", "# command (R = repository root):", "#   cd /tmp && export TMPDIR=/tmp",
         f"#   {a.cmd}", "#"]
    for k, name in SQ_DOC.items():
        L.append(f"# {k}: {name}")
    L.append("#")
    for kern, ctrs in sorted(by.items()):
        if not any(s in kern for s in a.kernels.split(",")):
            continue
        n = max(len(v) for v in ctrs.values())
        avg = {c: statistics.mean(v) for c, v in ctrs.items()}
        L.append(f"kernel: {kern[:160]}")
        L.append(f"  dispatches: {n}")
        for c in SQ_DOC:
            if c in avg:
                L.append(f"  {c}: {avg[c]:.0f}")
        # ratios of counters accumulated the same way (the absolute units of the
        # cycle counters are the hardware's; only the ratios are read here)
        if "SQ_ACTIVE_INST_VALU" in avg and "SQ_WAVE_CYCLES" in avg and avg["SQ_WAVE_CYCLES"] > 0:
            L.append(f"  VALU-issue cycles per resident wave-cycle: {avg['SQ_ACTIVE_INST_VALU'] / avg['SQ_WAVE_CYCLES']:.3f}")
        if "SQ_LDS_BANK_CONFLICT" in avg and "SQ_INSTS_LDS" in avg and avg["SQ_INSTS_LDS"] > 0:
            L.append(f"  LDS bank-conflict cycles per LDS instruction: {avg['SQ_LDS_BANK_CONFLICT'] / avg['SQ_INSTS_LDS']:.3f}")
        if "SQ_INSTS_VALU" in avg and "SQ_WAVES" in avg and avg["SQ_WAVES"] > 0:
            L.append(f"  VALU instructions per wave: {avg['SQ_INSTS_VALU'] / avg['SQ_WAVES']:.0f}")
    with open(a.out, "w") as f:
        f.write("\n".join(L) + "\n")
    print("\n".join(L))


def _copy_phase(a):
    import torch
    n = a.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.launches + 1):
        torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    print(f"copy bytes read = written = {n * 4}", flush=True)


def arnoldi(a):
    import torch
    from paper_2112_02211_amd import hps, problems as P

    prob = P.workload(a.workload)
    ctx = hps.Context.from_problem(prob, block_precs=("separable",), lambda_bucket=0.0)
    s, t = P.rhs_data(prob, ctx.nodes())
    s, t = torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda()
    _, st, _ = ctx.gmres(s, t, tol=prob.tol, restart=prob.restart)
    print(f"warm-up solve: {st['iters']} steps", flush=True)
    ctx.set_timing(True, every=1)
    ctx.arnoldi_times(reset=True)
    _, st, _ = ctx.gmres(s, t, tol=prob.tol, restart=prob.restart)
    at = ctx.arnoldi_times(reset=True)
    ctx.set_timing(False)
    print(f"arnoldi_update_launches: {at['update_launches']}", flush=True)
    print(f"arnoldi_update_algorithmic_bytes: {at['update_bytes']:.0f}", flush=True)
    print(f"arnoldi_update_ms: {at['update_ms']:.4f}", flush=True)
    _copy_phase(a)


def arnoldi_summary(a):
    """Traffic of the Arnoldi update pass over the second solve of `arnoldi`."""
    info = {}
    for line in open(a.run_log):
        if line.startswith("arnoldi_update_"):
            k, v = line.split(":", 1)
            info[k.strip()] = float(v)
    K = int(info["arnoldi_update_launches"])
    alg = info["arnoldi_update_algorithmic_bytes"]
    F = _counters(os.path.join(a.fetch, "run_counter_collection.csv"), "FETCH_SIZE")
    W = _counters(os.path.join(a.write, "run_counter_collection.csv"), "WRITE_SIZE")
    fu = _counters_of(os.path.join(a.fetch, "run_counter_collection.csv"), "FETCH_SIZE", "k_dcgs_update")
    wu = _counters_of(os.path.join(a.write, "run_counter_collection.csv"), "WRITE_SIZE", "k_dcgs_update")
    if len(fu) != 2 * K or len(wu) != 2 * K:
        raise ValueError(f"expected {2 * K} update dispatches, got {len(fu)}, {len(wu)}")
    med = lambda v: statistics.median(v[1:])
    ew_f, ew_w = med(_find(F, "MulFunctor<float>")), med(_find(W, "MulFunctor<float>"))
    copy_kib = a.copy_mib * 1024.0
    sf, sw = copy_kib / ew_f, copy_kib / ew_w
    tot = sum(fu[K:]) * 1024 * sf + sum(wu[K:]) * 1024 * sw
    cmd = f"python $R/paper_2112_02211_amd/profile_run.py arnoldi --workload {a.workload} --launches {a.launches}"
    L = [f"# HBM traffic of the Arnoldi update pass (k_dcgs_update), {a.workload} workload, one",
         "# left-preconditioned GMRES solve with the separable J^-1 (the second of two solves)",
         "#",
         "# commands (R = repository root; one counter per run):",
         "#   cd /tmp && export TMPDIR=/tmp",
         f"#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- {cmd}",
         f"#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o run -- {cmd}",
         f"#   python -m paper_2112_02211_amd.profile_run arnoldi-summary --workload {a.workload} "
         f"--launches {a.launches} --fetch <fetch dir> --write <write dir> --run-log <stdout of a run> --out <this file>",
         "#",
         f"# calibration: elementwise kernel dst = 2 src over {a.copy_mib} MiB float32",
         f"fetch_scale: {sf:.5f}",
         f"write_scale: {sw:.5f}",
         f"update_launches: {K}",
         f"update_algorithmic_bytes_total: {alg:.0f}",
         f"update_hbm_bytes_total: {tot:.0f}",
         f"traffic_over_algorithmic: {tot / alg:.4f}",
         f"kernel_source_sha256_16: {kernel_source_hash('k_dcgs_update')}",
         f"algorithmic_bytes_per_launch: {alg / K:.0f}",
         f"hbm_bytes_per_launch: {tot / K:.0f}"]
    # the separable J^-1 of the same solves (x in, y out, the neighbours' face
    # data read by the fused exchange): medians over its dispatches
    from paper_2112_02211_amd import problems as P
    prob = P.workload(a.workload)
    n1 = prob.p - 2
    nl = prob.n_elem[0] * prob.n_elem[1] * prob.n_elem[2]
    Nn = nl * (n1 ** 3 + 6 * n1 * n1)
    sk = [k for k in F if f"k_precond_sep<{prob.p}>" in k]
    if sk:
        fs, ws = _find(F, f"k_precond_sep<{prob.p}>"), _find(W, f"k_precond_sep<{prob.p}>")
        t_sep = statistics.median(f * 1024 * sf + w * 1024 * sw for f, w in zip(fs, ws))
        a_sep = 32.0 * Nn + 16.0 * nl * 6 * n1 * n1
        L += ["#", "# separable J^-1 (k_precond_sep) in the same solves, exchange fused",
              f"precond_sep_launches: {len(fs)}",
              f"precond_sep_algorithmic_bytes_per_launch: {a_sep:.0f}",
              f"precond_sep_hbm_bytes_per_launch: {t_sep:.0f}",
              f"precond_sep_traffic_over_algorithmic: {t_sep / a_sep:.4f}"]
    text = "\n".join(L) + "\n"
    open(a.out, "w").write(text)
    print(text)


def gemm(a):
    import numpy as np
    import torch
    from paper_2112_02211_amd import hps, problems as P

    prob = P.workload(a.workload)
    ctx = hps.Context.from_problem(prob, block_precs=("fp64", "fp32", "bf16"))
    rng = np.random.default_rng(0)
    X = torch.from_numpy(rng.standard_normal(a.rhs * ctx.N) + 1j * rng.standard_normal(a.rhs * ctx.N)).cuda()
    Y = torch.empty_like(X)
    for q in ("fp64", "fp32", "bf16"):
        shape = ctx.autotune(a.rhs, q, reps=1)
        for _ in range(a.launches + 1):
            ctx.precond(X, Y, prec=q)
        torch.cuda.synchronize()
        print(f"gemm {q}: shape {shape}, {a.launches + 1} launches", flush=True)
    print(f"gemm_algorithmic_flops: {8.0 * ctx.nl * ctx.nb * ctx.nb * a.rhs:.0f}", flush=True)


def gemm_summary(a):
    """Matrix-core counters of the block GEMM from one `gemm` run under
    rocprofv3 --pmc MfmaUtil MfmaFlopsF64 MfmaFlopsF32 MfmaFlopsBF16."""
    from paper_2112_02211_amd import problems as P
    prob = P.workload(a.workload)
    n1 = prob.p - 2
    nl = prob.n_elem[0] * prob.n_elem[1] * prob.n_elem[2]
    nb = 6 * n1 * n1
    alg = 8.0 * nl * nb * nb * a.rhs
    path = os.path.join(a.pmc_dir, "run_counter_collection.csv")
    rows = list(csv.DictReader(open(path)))
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        if "k_block_gemm" in r["Kernel_Name"]:
            per[(r["Kernel_Name"], int(r["Dispatch_Id"]))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    L = [f"# Matrix-core counters of the block GEMM of J^-1 on {a.rhs} right-hand sides, {a.workload}",
         f"# ({prob.n_elem[0]}x{prob.n_elem[1]}x{prob.n_elem[2]} leaves, p={prob.p}: {nl} blocks of {nb} x {nb})",
         "#",
         "# command (R = repository root):",
         "#   cd /tmp && export TMPDIR=/tmp",
         f"#   rocprofv3 --pmc MfmaUtil MfmaFlopsF64 MfmaFlopsF32 MfmaFlopsBF16 --output-format csv "
         f"-d <dir> -o run -- python "
         f"$R/paper_2112_02211_amd/profile_run.py gemm --workload {a.workload} --rhs {a.rhs} --launches {a.launches}",
         f"#   python -m paper_2112_02211_amd.profile_run gemm-summary --workload {a.workload} --rhs {a.rhs} "
         f"--launches {a.launches} --pmc-dir <that dir> --out <this file>",
         "#",
         f"# algorithmic flops per launch: 8 N_leaves n_b^2 k = {alg:.0f}",
         "# MfmaUtil: MFMA busy cycles / (active cycles x SIMDs), percent; MFMA flops = MOPS x 512",
         "# (medians over the dispatches after the first of each kernel)"]
    byk = collections.defaultdict(list)
    for (name, did), cnt in sorted(per.items(), key=lambda kv: kv[0][1]):
        byk[name].append({k: sum(v) for k, v in cnt.items()})
    for name, ds in byk.items():
        ds = ds[1:] if len(ds) > 1 else ds
        util = statistics.median(d.get("MfmaUtil", float("nan")) for d in ds)
        fl = {t: statistics.median(d.get(f"MfmaFlops{t}", 0.0) for d in ds) for t in ("F64", "F32", "BF16")}
        total = sum(fl.values())
        m = re.search(r"(k_block_gemm<[^>]*>)", name)
        short = m.group(1) if m else name.split("(")[0]
        L.append(f"{short}: MfmaUtil {util:.1f} %, MFMA flops per launch {total:.4g} "
                 f"(F64 {fl['F64']:.4g}, F32 {fl['F32']:.4g}, BF16 {fl['BF16']:.4g}), "
                 f"hardware / algorithmic {total / alg:.3f}, launches {len(ds)}")
    text = "\n".join(L) + "\n"
    open(a.out, "w").write(text)
    print(text)


def _counters(path, counter):
    """{kernel name: [values in dispatch order]} for one counter."""
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    d = collections.defaultdict(list)
    for r in rows:
        d[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return d


def _counters_of(path, counter, key):
    """Values of one counter, in dispatch order, over every kernel whose name
    contains key (the update pass has two kernels: the plain one and the one
    that ends a cycle with its closing reduction)."""
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter and key in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [float(r["Counter_Value"]) for r in rows]


def _find(d, key):
    hits = [v for k, v in d.items() if key in k]
    if len(hits) != 1:
        raise KeyError(f"{key}: {len(hits)} matching kernels")
    return hits[0]


def pmc_summary(a):
    """Traffic summary of the workload's kernels from a FETCH_SIZE and a
    WRITE_SIZE run of `run` (one warm-up plus `launches` dispatches per phase)."""
    from paper_2112_02211_amd import problems as P
    prob = P.workload(a.workload)
    p = prob.p
    n1 = p - 2
    nl = prob.n_elem[0] * prob.n_elem[1] * prob.n_elem[2]
    ni, nb = n1 ** 3, 6 * n1 * n1
    N = nl * (ni + nb)
    per = a.launches + 1
    F = _counters(os.path.join(a.fetch, "run_counter_collection.csv"), "FETCH_SIZE")
    W = _counters(os.path.join(a.write, "run_counter_collection.csv"), "WRITE_SIZE")
    med = lambda v: statistics.median(v[1:])          # drop the warm-up dispatch
    ew_f, ew_w = med(_find(F, "MulFunctor<float>")), med(_find(W, "MulFunctor<float>"))
    copy_kib = a.copy_mib * 1024.0
    sf, sw = copy_kib / ew_f, copy_kib / ew_w
    face = 16 * nl * nb
    ncp = {0: nb, 1: (nb + 1) // 2 * 2, 2: (nb + 3) // 4 * 4}
    el = {0: 16, 1: 8, 2: 4}
    L = [f"# HBM traffic of the hot-path kernels, {a.workload} workload",
         f"# ({prob.n_elem[0]}x{prob.n_elem[1]}x{prob.n_elem[2]} leaves, p={p}, N={N}; one launch "
         "applies the operator to one vector)",
         "#",
         "# commands (R = repository root; one counter per run):",
         "#   cd /tmp && export TMPDIR=/tmp",
         f"#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> "
         f"-o run -- python $R/paper_2112_02211_amd/profile_run.py --workload {a.workload} --launches {a.launches}"
         f"{' --iti' if a.iti else ''}",
         f"#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> "
         f"-o run -- python $R/paper_2112_02211_amd/profile_run.py --workload {a.workload} --launches {a.launches}"
         f"{' --iti' if a.iti else ''}",
         f"#   python -m paper_2112_02211_amd.profile_run pmc-summary --workload {a.workload} "
         f"--launches {a.launches}{' --iti' if a.iti else ''} --fetch <fetch dir> --write <write dir> --out <this file>",
         "#",
         f"# calibration: elementwise kernel dst = 2 src over {a.copy_mib} MiB float32 (reads and writes "
         f"{a.copy_mib << 20} bytes)",
         f"calib_fetch_size_kib: {ew_f:.0f}",
         f"calib_write_size_kib: {ew_w:.0f}",
         f"fetch_scale: {sf:.5f}",
         f"write_scale: {sw:.5f}",
         "# bytes = FETCH_SIZE[KiB] * 1024 * fetch_scale + WRITE_SIZE[KiB] * 1024 * write_scale",
         "# (medians over the timed dispatches of each phase)",
         "#"]
    fp = _find(F, f"k_precond_fused<{p}, 0>")
    wp = _find(W, f"k_precond_fused<{p}, 0>")
    if len(fp) != 2 * per or len(wp) != 2 * per:
        raise ValueError(f"expected {2 * per} FP64 preconditioner dispatches, got {len(fp)}, {len(wp)}")

    def line(name, f, w, alg):
        t = f * 1024 * sf + w * 1024 * sw
        L.append(f"# {name}: FETCH_SIZE {f:.0f} KiB, WRITE_SIZE {w:.0f} KiB per dispatch")
        L.append(f"{name}_hbm_bytes_per_launch: {t:.0f}")
        L.append(f"{name}_algorithmic_bytes_per_launch: {alg}")
        L.append(f"{name}_traffic_over_algorithmic: {t / alg:.4f}")
        return t

    # op_left runs first: its J^-1 dispatches carry the fused face exchange
    fused = line("fp64_fused_exchange", statistics.median(fp[1:per]), statistics.median(wp[1:per]),
                 16 * nl * nb * ncp[0] + 32 * N + face)
    line("fp64", statistics.median(fp[per + 1:]), statistics.median(wp[per + 1:]),
         16 * nl * nb * ncp[0] + 32 * N)
    for q, name in ((1, "fp32"), (2, "bf16")):
        line(name, med(_find(F, f"k_precond_fused<{p}, {q}>")), med(_find(W, f"k_precond_fused<{p}, {q}>")),
             el[q] * nl * nb * ncp[q] + 32 * N)
    sw_f, sw_w = _find(F, f"k_apply_sweep<{p},"), _find(W, f"k_apply_sweep<{p},")
    line("sweep", statistics.median(sw_f[1:]), statistics.median(sw_w[1:]),
         32 * N + 8 * nl * ni + face)
    bg = [k for k in F if "k_bgemv<false" in k]
    if bg:
        # the face-reduced operator's block product: R (16 nb^2 per leaf), f in, g out
        line("iti_block_product", med(_find(F, "k_bgemv<false")), med(_find(W, "k_bgemv<false")),
             16 * nl * nb * nb + 32 * nl * nb)
    L += ["#",
          "# the FP64 J^-1 with the fused exchange is the kernel the benchmark's roofline reports",
          f"kernel_source_sha256_16: {kernel_source_hash()}",
          f"hbm_bytes_per_launch: {fused:.0f}"]
    text = "\n".join(L) + "\n"
    open(a.out, "w").write(text)
    print(text)


def trace_summary(a):
    rows = list(csv.DictReader(open(a.stats)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    L = [f"# {a.title}", "#", "# command (R = repository root):",
         "#   cd /tmp && export TMPDIR=/tmp", f"#   {a.cmd}", "#",
         f"# {'kernel':70s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>10s} {'min_us':>9s} "
         f"{'max_us':>9s} {'pct':>6s}"]
    for r in rows[:a.rows]:
        name = r["Name"].replace("hps::(anonymous namespace)::", "").replace(
            "HIP_vector_type<double, 2u>", "double2").replace("HIP_vector_type<float, 2u>", "float2")[:70]
        L.append(f"  {name:70s} {r['Calls']:>6s} {float(r['TotalDurationNs']) / 1e6:10.2f} "
                 f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:9.2f} "
                 f"{float(r['MaxNs']) / 1e3:9.2f} {100 * float(r['TotalDurationNs']) / tot:6.2f}")
    text = "\n".join(L) + "\n"
    open(a.out, "w").write(text)
    print(text)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", nargs="?", default="run",
                    choices=("run", "pmc-summary", "trace-summary", "arnoldi", "arnoldi-summary", "gemm",
                             "gemm-summary", "sep", "sq-summary"))
    ap.add_argument("--workload", default="bumps_8x8x8_p10")
    ap.add_argument("--launches", type=int, default=4)
    ap.add_argument("--iti", action="store_true",
                    help="run: also the face-reduced operator (builds the exact ItI maps)")
    ap.add_argument("--lambda-bucket", type=float, default=0.0,
                    help="run: lambda grid spacing (times kappa^2) of shared blocks; 0: one per leaf")
    ap.add_argument("--copy-mib", type=int, default=COPY_MIB)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--stats")
    ap.add_argument("--run-log")
    ap.add_argument("--rhs", type=int, default=64)
    ap.add_argument("--pmc-dir")
    ap.add_argument("--out")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--title", default="rocprofv3 kernel statistics")
    ap.add_argument("--rows", type=int, default=24)
    ap.add_argument("--kernels", default="k_apply_sweep,k_precond_sep",
                    help="sq-summary: comma-separated kernel name substrings")
    a = ap.parse_args()
    {"run": run, "pmc-summary": pmc_summary, "trace-summary": trace_summary, "arnoldi": arnoldi,
     "arnoldi-summary": arnoldi_summary, "gemm": gemm, "gemm-summary": gemm_summary, "sep": sep,
     "sq-summary": sq_summary}[a.mode](a)


if __name__ == "__main__":
    main()
