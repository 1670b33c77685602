"""Benchmark: one step = the whole hot path on the F2 workload of the
paper's Table 2 family at n = 2^22 (GKR prove + verify of the F2 circuit,
12,582,911 gates, seed 2) plus the F2 sum-check on a 2^26-entry vector
(prove + verify, seed 2).  Inputs are resident in HBM before timing.

value = GKR prover gates/s = gates (inputs included, as Table 2 counts
them) / mean time of gkr_prove, which includes device evaluation, every
sum-check round and the transcript copy to the host.

Further legs (each with its own flag to skip it): the F2 circuit at n = 2^10
and MatMult at N = 256; a batch of 64 uneven proofs against the same proofs
one by one; a proof server under Poisson arrivals against the same requests
proved one by one; Table 2's F0-based circuits; the out-of-core memory
strategies under device budgets; Table 3's non-interactive F2 protocol; and
the CPU oracle on bounded samples at one thread and at every host thread.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Modular products per second the chip can issue: 256 CUs x 4 SIMDs, one
# wave64 VALU instruction per SIMD every 4 cycles at 2.4 GHz (3.93e13 32-bit
# lane operations/s), 21 VALU instructions per product of the field module.
ALU_PEAK_MULMOD = 256 * 4 * 64 / 4 * 2.4e9 / 21


def kernel_source_hash():
    """Hash of every kernel and launch-planning source: a counter summary
    taken on other sources no longer describes the kernels."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1202_1350_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


# Step kinds in the order of the StepKind enum: the profiling class
# "step_<kind>" is the kernel k_step_one<kind index, ...>.
STEP_KINDS = ["eval", "start", "eq", "p", "w", "fold", "lt", "line", "sge", "end", "wagg",
              "wt0", "wt", "wtail", "ptail", "load", "wa0", "finish", "wsmall", "top", "lfold"]


def rocprof_kernel_name(cls):
    """How rocprofv3 names the kernels of a profiling class (the
    single-proof step kernels, k_step_one<kind, *, *>: some kinds have one
    kernel per gate mix and phase; other classes are returned unchanged)."""
    if cls.startswith("step_") and cls[5:] in STEP_KINDS:
        return f"void gkr::k_step_one<{STEP_KINDS.index(cls[5:])}u, *, *>(gkr::StepDesc)"
    return cls


def kernel_matches(name, cls):
    """Whether rocprofv3's kernel name is one of cls's kernels."""
    pat = rocprof_kernel_name(cls)
    if "*" not in pat:
        return name == pat
    return name.startswith(pat.split("*")[0])


def traffic_path(cls):
    return os.path.join(ROOT, "profiles", f"{cls}_f2_n2p22_traffic.txt")


def measured_traffic(cls):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources (else None)."""
    path = traffic_path(cls)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _pmc_rows(d, counter):
    """(kernel name, value) per dispatch from a rocprofv3 --pmc csv."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    rows = []
    for f in files:
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") == counter:
                rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def traffic_summary(fetch_dir, write_dir, cls, copy_bytes, command):
    """Text summary of HBM traffic per launch of one kernel from two
    rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each
    scaled by what the same counter reads for the calibration copy (the
    largest device-to-device blit, of copy_bytes read and written)."""
    name = rocprof_kernel_name(cls)
    out = [f"# HBM traffic of {name} (class {cls}), F2 GKR n=2^22, seed 2",
           f"# command: {command}"]
    per = {}
    for label, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = _pmc_rows(d, counter)
        copies = [v for k, v in rows if "copyBuffer" in k]
        kern = [v for k, v in rows if kernel_matches(k, cls)]
        if not copies or not kern:
            raise SystemExit(f"{counter}: calibration copy or kernel {name} missing")
        cal = max(copies) * 1024.0
        factor = copy_bytes / cal
        per[label] = sum(kern) / len(kern) * 1024.0 * factor
        out += [f"{label}_counter: {counter}",
                f"{label}_dispatches: {len(kern)}",
                f"{label}_calibration_copy_counter_bytes: {cal:.0f}",
                f"{label}_calibration_factor: {factor:.4f}",
                f"{label}_bytes_per_launch: {per[label]:.0f}"]
    out += [f"copy_bytes: {copy_bytes}",
            f"hbm_bytes_per_launch: {per['fetch'] + per['write']:.0f}",
            f"kernel_source_hash: {kernel_source_hash()}"]
    return "\n".join(out) + "\n"


TUNE_FILE = os.path.join(ROOT, "paper_1202_1350_amd", "tune_table.txt")


def load_tune_table(G, path):
    """Install a saved launch-shape table if it was tuned on the current
    kernel sources; returns True if installed."""
    if not os.path.exists(path):
        return False
    vals = dict(l.split(":", 1) for l in open(path) if ":" in l and not l.startswith("#"))
    if vals.get("kernel_source_hash", "").strip() != kernel_source_hash():
        return False
    G.gkr_tune_set(bytes.fromhex(vals["table"].strip()))
    return True


def save_tune_table(G, path, note):
    with open(path, "w") as f:
        f.write("# launch shapes chosen by gkr_autotune (" + note + ")\n")
        f.write(f"kernel_source_hash: {kernel_source_hash()}\n")
        f.write(f"table: {G.gkr_tune_get().hex()}\n")


def note(*a):
    """A progress line on stderr, one per leg of the benchmark."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_info():
    """Host CPU model (lscpu) and thread count."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def oracle_threads():
    """Every host thread, at most 16 (the GPU machine's CPU share)."""
    return max(1, min(16, os.cpu_count() or 1))


def cpu_baseline(W, np):
    """The oracle (plain C, the tests' reference) on the host cores, on
    bounded samples of the benchmark workloads: the F2 GKR circuit (C2a's
    construction) at 2^20 inputs on every thread and 2^17 on one, the F2
    sum-check (C2b's) at 2^24 and 2^21, and MatMult (C3's) at N = 64 and 32.
    The headline sample is F2 at 2^20 on every thread."""
    from oracle import oracle as O
    O.build(force=False)
    T = oracle_threads()
    res = {"host": cpu_info(), "samples": []}

    def run(name, threads, gates, fn, unit="gates/s"):
        note("oracle:", name, f"threads={threads}")
        O.set_threads(threads)
        t = time.perf_counter()
        fn()
        dt = time.perf_counter() - t
        res["samples"].append({"workload": name, "threads": threads, "seconds": dt,
                               "value": gates / dt, "unit": unit})
        return dt

    circ20, x20, _ = W.c2_f2(20)
    circ17, x17, _ = W.c2_f2(17)
    head = run("F2 GKR prove, n=2^20, seed 2", T, circ20.gates, lambda: O.prove(circ20, x20, 2))
    run("F2 GKR prove, n=2^17, seed 2", 1, circ17.gates, lambda: O.prove(circ17, x17, 2))
    a24, a21 = W.f2sc_vector(1 << 24, 2), W.f2sc_vector(1 << 21, 2)
    run("F2 sum-check prove, n=2^24, seed 2", T, 1 << 24, lambda: O.f2sc_prove(a24, 2), "values/s")
    run("F2 sum-check prove, n=2^21, seed 2", 1, 1 << 21, lambda: O.f2sc_prove(a21, 2), "values/s")
    for N, th in ((64, T), (32, 1)):
        c, x = W.matmult_circuit(N), W.matmult_inputs(N, 3)
        run(f"MatMult GKR prove, N={N}, seed 3", th, c.gates, lambda: O.prove(c, x, 3))
    # batched workload: the first eight proofs of the 64-proof batch (seed 4),
    # one after another; serving: one proof of each request type
    mix = W.batch_mix(4, 64)[:8]
    t = time.perf_counter()
    O.set_threads(T)
    for _, c, x, sd in mix:
        O.prove(c, x, sd)
    dt = time.perf_counter() - t
    res["samples"].append({"workload": "first 8 proofs of the 64-proof batch (seed 4), summed", "threads": T,
                           "seconds": dt, "value": sum(c.gates for _, c, _, _ in mix) / dt, "unit": "gates/s"})
    for name, c, x in (("F2 n=2^14", W.f2_circuit(1 << 14), W.f2_inputs(1 << 14, 64)),
                       ("F2 n=2^18", W.f2_circuit(1 << 18), W.f2_inputs(1 << 18, 68)),
                       ("MatMult N=64", W.matmult_circuit(64), W.matmult_inputs(64, 64)),
                       ("PM text 2^16", W.pm_circuit(1 << 16), W.pm_inputs(1 << 16, 66)[0])):
        run(f"serving request type {name}, one proof", T, c.gates, lambda c=c, x=x: O.prove(c, x, 5))
    # the unverifiable computations the paper compares against (numpy, one pass)
    t = time.perf_counter()
    _ = int((x20.astype(np.float64) ** 2).sum())
    res["direct_f2_2p20_s"] = time.perf_counter() - t
    res["headline"] = {"value": circ20.gates / head, "unit": "gates/s", "cores": T, "kind": "oracle",
                       "sample": f"one full oracle proof of the F2 circuit at n=2^20 ({circ20.gates} gates, "
                                 f"seed 2) in {head:.2f} s on {T} threads; the benchmark circuit is n=2^22",
                       **cpu_info()}
    return res


def config_leg(G, W, np, torch, make, name, reps):
    """One benchmark configuration proved and verified with its inputs
    resident: mean prove time over reps after a warm-up proof, median of
    five verifications."""
    circ, x, seed = make()
    gc = G.Circuit.from_workload(circ)
    xt = torch.from_numpy(x.view(np.int64)).cuda().view(torch.uint64)
    m, _ = G.gkr_prove(gc, xt, seed, want_chals=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        G.gkr_prove(gc, xt, seed, want_chals=False)
    dt = (time.perf_counter() - t) / reps
    tv = []
    for _ in range(5):
        t = time.perf_counter()
        ok = G.gkr_verify(gc, xt, seed, m)[0]
        tv.append(time.perf_counter() - t)
        if not ok:
            raise SystemExit(f"verifier rejected an honest transcript ({name})")
    return {"workload": name, "gates": circ.gates, "rounds": gc.rounds, "msgs": gc.n_msgs,
            "prove_ms": dt * 1e3, "gates_per_s": circ.gates / dt, "proofs_per_s": 1.0 / dt,
            "verify_ms": 1e3 * sorted(tv)[2], "accepted": True}


def size_sweep(G, W, np, torch):
    """Prover gates/s against input size (the analogue of the paper's
    Fig. 5: speedups grow with the input as fixed costs amortise): F2 at
    n = 2^10 .. 2^22 and MatMult at N = 16 .. 256, inputs resident, mean of
    five proofs after a warm-up."""
    out = []
    cases = [("F2", n, lambda n=n: (W.f2_circuit(n), W.f2_inputs(n, 60 + n))) for n in
             (1 << 10, 1 << 12, 1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22)]
    cases += [("MatMult", N, lambda N=N: (W.matmult_circuit(N), W.matmult_inputs(N, 60 + N)))
              for N in (16, 32, 64, 128, 256)]
    for kind, size, make in cases:
        circ, x = make()
        gc = G.Circuit.from_workload(circ)
        xt = torch.from_numpy(x.view(np.int64)).cuda().view(torch.uint64)
        G.gkr_prove(gc, xt, 5, want_chals=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            G.gkr_prove(gc, xt, 5, want_chals=False)
        dt = (time.perf_counter() - t) / 5
        out.append({"circuit": kind, "size": size, "gates": circ.gates, "rounds": gc.rounds,
                    "prove_ms": dt * 1e3, "gates_per_s": circ.gates / dt})
        del gc, xt
    return out


# Table 2's GPU prover times in seconds (the paper's GPU; context only).
TABLE2_GPU_PROVE_S = {"F0": 128.5, "PM": 38.9, "MatMult": 39.6}


def table2_leg(G, W, np, torch, reps, with_oracle, keep=()):
    """Table 2's other three rows at its sizes, on circuits built on the F0
    (Fermat) stage: F0 of 2^21 values, pattern matching with the F0 count on
    a 2^19 text (q = 8), MatMult with the C = AB check (N = 256).  Prove and
    verify times with inputs resident; the oracle on a bounded sample of
    each circuit family.  Returns the records and, for the names in keep,
    (handle, inputs, seed, transcript) for the out-of-core leg."""
    from oracle import oracle as O
    fams = (("F0", W.f1_f0, lambda: (W.f0_circuit(1 << 12), W.f0_inputs(1 << 12, 6), 6), "F0 n=2^12"),
            ("PM", W.f1_pm_f0, lambda: (W.pm_f0_circuit(1 << 12, 8), W.pm_inputs(1 << 12, 7, 8)[0], 7),
             "PM-F0 text 2^12, q=8"),
            ("MatMult", W.f1_matmult_check,
             lambda: (W.matmult_check_circuit(16), W.matmult_check_inputs(16, 8)[0], 8), "MatMult-check N=16"))
    out, kept = {}, {}
    for name, make, small, small_name in fams:
        circ, x, seed = make()
        gc = G.Circuit.from_workload(circ)
        xt = torch.from_numpy(x.view(np.int64)).cuda().view(torch.uint64)
        m, _ = G.gkr_prove(gc, xt, seed, want_chals=False)  # scratch and graph set up
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            G.gkr_prove(gc, xt, seed, want_chals=False)
        dt = (time.perf_counter() - t) / reps
        t = time.perf_counter()
        ok = G.gkr_verify(gc, xt, seed, m)[0]
        tv = time.perf_counter() - t
        rec = {"circuit": circ.name, "gates": circ.gates, "depth": circ.depth, "output": int(m[0]),
               "accepted": bool(ok), "prove_ms": dt * 1e3, "gates_per_s": circ.gates / dt,
               "verify_ms": tv * 1e3, "paper_gpu_prove_s": TABLE2_GPU_PROVE_S[name]}
        if with_oracle:
            sc, sx, ss = small()
            O.build(force=False)
            threads = oracle_threads()
            O.set_threads(threads)
            t = time.perf_counter()
            O.prove(sc, sx, ss)
            to = time.perf_counter() - t
            rec["oracle"] = {"gates_per_s": sc.gates / to, "cores": threads,
                             "sample": f"{small_name} ({sc.gates} gates) in {to:.2f} s"}
        out[name] = rec
        if name in keep:
            kept[name] = (gc, circ.name, xt, seed, m, dt)
        del gc, xt, circ, x
    return out, kept


MEM_NAMES = {0: "resident (no copying)", 1: "copy once per layer", 2: "copy every message"}


def ooc_leg(G, np, torch, kept, reps):
    """Out-of-core proofs (Sec. 5.1.2, 5.1.3): each circuit proved under
    device budgets of 1/4 and 1/8 of what its resident proof needs (the
    first memory strategy that fits), and F0 in both strategies, against the
    resident proof; transcripts must be bit-equal."""
    out = {}
    for name, (gc, cname, xt, seed, m_res, t_res) in kept.items():
        need = {k: gc.memory_need(k) for k in (0, 1, 2)}
        runs = []
        plans = [("budget 1/4", G.GKR_MEM_AUTO, need[0][0] // 4), ("budget 1/8", G.GKR_MEM_AUTO, need[0][0] // 8)]
        if name == "F0":
            plans += [("forced", G.GKR_MEM_LAYER, 0), ("forced", G.GKR_MEM_MESSAGE, 0)]
        for label, mode, budget in plans:
            chosen = gc.set_memory(mode, budget)
            m, _ = G.gkr_prove(gc, xt, seed, want_chals=False)  # scratch set up
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                G.gkr_prove(gc, xt, seed, want_chals=False)
            dt = (time.perf_counter() - t) / reps
            runs.append({"what": label, "device_budget_bytes": budget, "mode": MEM_NAMES[chosen],
                         "device_bytes": need[chosen][0], "host_bytes": need[chosen][1],
                         "prove_ms": dt * 1e3, "slowdown_vs_resident": dt / t_res,
                         "bit_exact_vs_resident": bool(np.array_equal(m, m_res))})
            print(f"out of core {name} {label} {MEM_NAMES[chosen]}: {dt * 1e3:.1f} ms "
                  f"({dt / t_res:.1f}x resident)", file=sys.stderr, flush=True)
        gc.set_memory(G.GKR_MEM_RESIDENT)
        rec = {"circuit": cname, "resident_prove_ms": t_res * 1e3,
               "need_bytes": {MEM_NAMES[k]: {"device": v[0], "host": v[1]} for k, v in need.items()},
               "runs": runs}
        layer = [r for r in runs if r["mode"] == MEM_NAMES[1]]
        msg = [r for r in runs if r["mode"] == MEM_NAMES[2]]
        if layer and msg:
            rec["message_vs_layer"] = msg[-1]["prove_ms"] / layer[-1]["prove_ms"]
            rec["paper_message_vs_layer"] = "< 3x (preliminary, Sec. 5.1.3)"
        out[name] = rec
    return out


# Table 3 (non-interactive F2, n = 25 million): the paper's (v space,
# proof length, GPU prover seconds) per row; h here is the admissible row
# length nearest the paper's (h must divide (p - 1) / 2).
TABLE3 = [(5005, "39.1 KB / 78.1 KB", 2.901), (2475, "78.2 KB / 39.1 KB", 1.872),
          (1287, "156.5 KB / 19.5 KB", 1.154), (585, "313.2 KB / 9.8 KB", 0.909),
          (45, "1953.1 KB / 0.78 KB", 0.357)]


def table3_leg(G, np, torch, reps, with_oracle):
    """The non-interactive F2 protocol on n = 25 million values in [0, 2^16)
    (seed 25) for Table 3's space / proof-length tradeoffs: prove and verify
    times with the values resident in HBM, and the oracle on one grid."""
    n = 25_000_000
    rng = np.random.default_rng(25)
    a = rng.integers(0, 1 << 16, n).astype(np.uint64)
    at = torch.from_numpy(a.view(np.int64)).cuda().view(torch.uint64)
    out = []
    for h, tradeoff, paper_s in TABLE3:
        m = G.nif2_prove(at, h)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            G.nif2_prove(at, h)
        dt = (time.perf_counter() - t) / reps
        t = time.perf_counter()
        ok, _ = G.nif2_verify(at, h, 1, m)
        tv = time.perf_counter() - t
        v = -(-n // h)
        out.append({"h": h, "v": v, "proof_words": 2 * h, "paper_tradeoff": tradeoff,
                    "prove_ms": dt * 1e3, "values_per_s": n / dt, "verify_ms": tv * 1e3,
                    "accepted": bool(ok), "paper_gpu_prove_s": paper_s})
    res = {"n": n, "data": "uniform in [0, 2^16), seed 25", "rows": out}
    if with_oracle:
        from oracle import oracle as O
        O.build(force=False)
        threads = max(1, min(16, os.cpu_count() or 1))
        O.set_threads(threads)
        h, v = 1287, 64
        t = time.perf_counter()
        O.nif2_prove(a[:h * v], h)
        to = time.perf_counter() - t
        res["oracle"] = {"values_per_s": h * v / to, "cores": threads,
                         "sample": f"the {h * v} first values on a {v} x {h} grid in {to:.2f} s "
                                   "(direct Lagrange evaluation, O(h^2 v))"}
    return res


def launch_roofline(prof_entry, alu_peak, kernel):
    """HBM and ALU fractions of a kernel class from its profiled launches
    (total ms, launches, algorithmic bytes, algorithmic products)."""
    ms, n, by, mo = prof_entry
    if not n or ms <= 0:
        return None
    gbs = by / (ms * 1e-3) / 1e9
    mps = mo / (ms * 1e-3)
    fh, fa = gbs / HBM_PEAK_GBS, mps / alu_peak
    return {"kernel": kernel, "launches": n, "avg_launch_us": ms * 1e3 / n,
            "algorithmic_bytes_per_launch": by / n, "algorithmic_products_per_launch": mo / n,
            "hbm": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fh},
            "alu": {"achieved": mps / 1e9, "peak": alu_peak / 1e9, "unit": "Gmulmod/s", "frac": fa},
            "bound": "alu" if fa > fh else "hbm"}


def batch_leg(G, W, np, torch, reps, tune, alu_peak):
    """64 uneven proofs (F2 n log-uniform in [2^12, 2^20], PM text in
    [2^14, 2^18], seed 4): the plain path proves them one by one (one
    gkr_prove each, that proof's own launches replayed from its graph; no
    launch fuses proofs), the batched path in one launch per step (graph
    replay).  Both must give the same transcripts.  Launch shapes are tuned
    on these circuits for this leg and restored afterwards."""
    mix = W.batch_mix(4, 64)
    circs = [G.Circuit.from_workload(c) for _, c, _, _ in mix]
    xs = [torch.from_numpy(x.view(np.int64)).cuda().view(torch.uint64) for _, _, x, _ in mix]
    seeds = [sd for _, _, _, sd in mix]
    gates = sum(c.gates for c in circs)
    saved = G.gkr_tune_get()
    tune_s = None
    try:
        if tune:
            t = time.perf_counter()
            G.gkr_autotune(circs, xs, reps=1)
            tune_s = time.perf_counter() - t
        plain = [G.gkr_prove(c, x, sd, want_chals=False)[0] for c, x, sd in zip(circs, xs, seeds)]
        batched = G.gkr_batch_prove(circs, xs, seeds)
        same = all(np.array_equal(a, b) for a, b in zip(plain, batched))
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            for c, x, sd in zip(circs, xs, seeds):
                G.gkr_prove(c, x, sd, want_chals=False)
        t_plain = (time.perf_counter() - t) / reps
        t = time.perf_counter()
        for _ in range(reps):
            G.gkr_batch_prove(circs, xs, seeds)
        t_batch = (time.perf_counter() - t) / reps
        # the batched kernel's launches timed one by one (outside the timed region)
        G.gkr_profile_read()
        G.gkr_profile_enable(1)
        G.gkr_batch_prove(circs, xs, seeds)
        G.gkr_profile_enable(0)
        prof = G.gkr_profile_read()
    finally:
        G.gkr_tune_set(saved)
    return {"workload": "64 uneven proofs: F2 n=2^[12,20], PM text 2^[14,18] (seed 4)",
            "proofs": len(circs), "gates": gates, "bit_exact_batched_vs_plain": same,
            "plain_ms": t_plain * 1e3, "batched_ms": t_batch * 1e3,
            "plain_path": "one gkr_prove per proof, each replaying its own graph of launches",
            "plain_gates_per_s": gates / t_plain, "batched_gates_per_s": gates / t_batch,
            "batched_proofs_per_s": len(circs) / t_batch, "speedup": t_plain / t_batch,
            "launch_shapes": "tuned on this batch for this leg (then restored)" if tune else "defaults",
            "autotune_seconds": tune_s,
            "roofline": launch_roofline(prof.get("batch_step", (0, 0, 0, 0)), alu_peak,
                                        "gkr::k_step_jobs(gkr::JobEntry const*, unsigned int)")}


def serve_requests(W, np, total, seed=5):
    """Poisson proof requests (seed 5, purpose 5): type uniform over F2 (n =
    2^u rounded up to 16 sizes per octave, u uniform in [14, 22]), MatMult
    (N in {64, 128, 256}) and PM (text 2^16, pattern 8); per request (kind,
    size, proof seed, unit exponential gap)."""
    import math
    draws = W.splitmix64(seed, 5, 4 * total)
    reqs = []
    for k in range(total):
        kind = int(draws[4 * k] % np.uint64(3))
        v01 = float(draws[4 * k + 1] >> np.uint64(11)) / float(1 << 53)
        if kind == 0:
            e = 14.0 + 8.0 * v01
            g = 1 << (int(e) - 4)
            n = min(1 << 22, int(math.ceil(2.0 ** e / g)) * g)
            kind, size = "F2", n
        elif kind == 1:
            kind, size = "MM", (64, 128, 256)[int(draws[4 * k + 1] % np.uint64(3))]
        else:
            kind, size = "PM", 1 << 16
        gap = -math.log(1.0 - float(draws[4 * k + 2] >> np.uint64(11)) / float(1 << 53))
        reqs.append((kind, size, int(draws[4 * k + 3] >> np.uint64(8)), gap))
    return reqs


def serve_leg(G, W, np, n_req, n_sat, rates, alu_peak):
    """The Poisson request mix (serve_requests) on a continuous-batching
    server (32 slots, 32 GiB budget).  The circuit of every distinct shape
    is created before timing, as a service loads its circuits.  First the
    closed-loop saturation rate (n_sat requests submitted at once), then the
    same n_sat requests proved one by one with gkr_prove (the plain path;
    transcripts must be bit-equal to the served ones), then open-loop
    arrivals at the given fractions of saturation, n_req requests per point,
    the first 10% of each point warm-up.  Latency runs from the scheduled
    arrival to completion."""
    total = n_sat + n_req * len(rates)
    reqs = serve_requests(W, np, total)
    shapes = {}
    for kind, size, _, _ in reqs:
        if (kind, size) in shapes:
            continue
        if kind == "F2":
            c, x = W.f2_circuit(size), W.f2_inputs(size, 50 + size)
        elif kind == "MM":
            c, x = W.matmult_circuit(size), W.matmult_inputs(size, 50 + size)
        else:
            c, x = W.pm_circuit(size), W.pm_inputs(size, 50 + size)[0]
        shapes[(kind, size)] = (G.Circuit.from_workload(c), x, c.gates)

    def shape(kind, size):
        return shapes[(kind, size)]

    srv = G.Server(32 << 30, 32)
    try:
        ids = [srv.submit(c, x, 1) for c, x, _ in shapes.values()]  # every shape's scratch pool warmed
        while ids:
            ids = [r for r in ids if not srv.poll(r)[0]]
        # closed loop: all requests at once
        sat_reqs = reqs[:n_sat]
        sat_gates = sum(shape(k, sz)[2] for k, sz, _, _ in sat_reqs)
        t0 = time.perf_counter()
        ids = [srv.submit(shape(k, sz)[0], shape(k, sz)[1], sd) for k, sz, sd, _ in sat_reqs]
        served, pending = {}, set(ids)
        while pending:
            for r in list(pending):
                done, m, _ = srv.poll(r)
                if done:
                    served[r] = m
                    pending.discard(r)
        t_sat = time.perf_counter() - t0
        sat = n_sat / t_sat
        # the same requests, one gkr_prove each (host inputs, as the server takes them)
        for c, x, _ in shapes.values():
            G.gkr_prove(c, x, 1, want_chals=False)  # each circuit's scratch and graph set up
        t0 = time.perf_counter()
        alone = [G.gkr_prove(shape(k, sz)[0], shape(k, sz)[1], sd, want_chals=False)[0]
                 for k, sz, sd, _ in sat_reqs]
        t_plain = time.perf_counter() - t0
        exact = all(np.array_equal(served[r], a) for r, a in zip(ids, alone))
        points = []
        for pi, frac in enumerate(rates):
            rate = frac * sat
            part = reqs[n_sat + n_req * pi: n_sat + n_req * (pi + 1)]
            arrivals = np.cumsum([gap / rate for _, _, _, gap in part])
            warm = len(part) // 10
            t0 = time.perf_counter()
            sched, done_at, gates_of = {}, {}, {}
            k = 0
            pending = set()
            while k < len(part) or pending:
                now = time.perf_counter() - t0
                while k < len(part) and arrivals[k] <= now:
                    kind, sz, sd, _ = part[k]
                    c, x, g = shape(kind, sz)
                    rid = srv.submit(c, x, sd)
                    sched[rid] = (k, arrivals[k])
                    gates_of[rid] = g
                    pending.add(rid)
                    k += 1
                for rid in list(pending):
                    if srv.poll(rid)[0]:
                        done_at[rid] = time.perf_counter() - t0
                        pending.discard(rid)
                if k < len(part) and not pending:
                    time.sleep(max(0.0, min(0.001, arrivals[k] - (time.perf_counter() - t0))))
            # measurement window: after the warm-up requests have arrived
            w0 = arrivals[warm] if warm < len(arrivals) else 0.0
            in_win = [r for r in done_at if sched[r][0] >= warm]
            span = max(done_at[r] for r in in_win) - w0
            lats = sorted(done_at[r] - sched[r][1] for r in in_win)
            points.append({"rate_frac_of_saturation": frac, "offered_proofs_per_s": rate,
                           "requests_measured": len(in_win),
                           "proofs_per_s": len(in_win) / span,
                           "gates_per_s": sum(gates_of[r] for r in in_win) / span,
                           "p50_ms": 1e3 * lats[len(lats) // 2],
                           "p99_ms": 1e3 * lats[min(len(lats) - 1, int(0.99 * len(lats)))]})
            print(f"serve point {frac:.2f}x: {points[-1]['proofs_per_s']:.1f} proofs/s, "
                  f"p50 {points[-1]['p50_ms']:.1f} ms, p99 {points[-1]['p99_ms']:.1f} ms",
                  file=sys.stderr, flush=True)
        # the server's launches timed one by one (outside the timed region)
        G.gkr_profile_read()
        G.gkr_profile_enable(1)
        ids = [srv.submit(shape(k, sz)[0], shape(k, sz)[1], sd) for k, sz, sd, _ in reqs[:min(100, n_sat)]]
        while ids:
            ids = [r for r in ids if not srv.poll(r)[0]]
        G.gkr_profile_enable(0)
        prof = G.gkr_profile_read()
    finally:
        srv.close()
    kinds = {}
    for kind, size in shapes:
        kinds.setdefault(kind, set()).add(size)
    return {"workload": "Poisson mix of F2 n=2^u (u uniform in [14,22], 16 sizes per octave), MatMult "
                        "N in {64,128,256}, PM text 2^16 (seed 5); 32 slots, 32 GiB budget",
            "distinct_shapes": {k: len(v) for k, v in kinds.items()},
            "requests_per_point": n_req, "warmup_fraction": 0.1,
            "closed_loop_requests": n_sat, "closed_loop_proofs_per_s": sat,
            "closed_loop_gates_per_s": sat_gates / t_sat,
            "plain_same_requests": {"path": "one gkr_prove per request, host inputs",
                                    "proofs_per_s": n_sat / t_plain, "gates_per_s": sat_gates / t_plain},
            "served_vs_plain_gates_per_s": t_plain / t_sat,
            "bit_exact_served_vs_alone": exact,
            "points": points,
            "roofline": launch_roofline(prof.get("serve_step", (0, 0, 0, 0)), alu_peak,
                                        "gkr::k_step_table(gkr::JobTable)")}


def mulmod_rate(G, torch, dev):
    """Products per second of the device field module: 2^24 independent
    chains of 256 dependent products each (best of three)."""
    n = 1 << 24
    g = torch.Generator().manual_seed(7)
    a = torch.randint(0, (1 << 61) - 1, (n,), generator=g, dtype=torch.int64).to(dev).view(torch.uint64)
    b = torch.randint(0, (1 << 61) - 1, (n,), generator=g, dtype=torch.int64).to(dev).view(torch.uint64)
    out = torch.empty_like(a)
    G.gkr_field_op(4, a, b, out)
    best = None
    for _ in range(3):
        t = time.perf_counter()
        G.gkr_field_op(4, a, b, out)  # synchronises
        dt = time.perf_counter() - t
        best = dt if best is None else min(best, dt)
    return n * 256 / best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log-n", type=int, default=22)
    ap.add_argument("--f2sc-log-n", type=int, default=26)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the F2 n=2^10 (seed 1) and MatMult N=256 (seed 3) legs")
    ap.add_argument("--no-ooc", action="store_true",
                    help="skip the out-of-core memory strategies (F0 2^21, MatMult check N=256)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-table2", action="store_true",
                    help="skip the F0, PM-F0 and MatMult-check circuits at Table 2's sizes")
    ap.add_argument("--no-table3", action="store_true",
                    help="skip the non-interactive F2 protocol at Table 3's size")
    ap.add_argument("--autotune", choices=["auto", "off", "force"], default="auto",
                    help="auto: load the saved launch-shape table if it matches the kernel "
                         "sources, else tune on the benchmark circuit; off: default shapes; "
                         "force: tune")
    ap.add_argument("--write-tune", metavar="PATH", help="save the launch-shape table used")
    ap.add_argument("--serve-requests", type=int, default=1000, help="requests per rate point")
    ap.add_argument("--serve-points", type=int, default=8,
                    help="rate points, geometric from 0.1x to 1.5x saturation")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also copy a buffer of this size device to device (the "
                         "known-size kernel that scales the HBM counters)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the HBM traffic summary of two rocprofv3 --pmc runs and exit")
    ap.add_argument("--kernel", default="step_wt0", help="profiling class for --traffic-summary")
    ap.add_argument("--command", default="", help="command line recorded in --traffic-summary")
    args = ap.parse_args()
    if args.traffic_summary:
        sys.stdout.write(traffic_summary(args.traffic_summary[0], args.traffic_summary[1],
                                         args.kernel, args.copy_calibration_mib << 20,
                                         args.command))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "sharding is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1202_1350_amd as G
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    circ, x, seed = W.c2_f2(args.log_n)
    a, fseed = W.c2_f2sc(args.f2sc_log_n)
    gc = G.Circuit.from_workload(circ)
    xt = torch.from_numpy(x.view(np.int64)).to(dev).view(torch.uint64)
    at = torch.from_numpy(a.view(np.int32)).to(dev).view(torch.uint32)
    torch.cuda.synchronize()
    tune = {"mode": args.autotune}
    G.gkr_tune_set(None)
    if args.autotune == "auto" and load_tune_table(G, TUNE_FILE):
        tune["source"] = os.path.relpath(TUNE_FILE, ROOT)
    elif args.autotune != "off":
        t = time.perf_counter()
        G.gkr_autotune([gc], [xt], reps=2)
        tune.update(source="tuned now on the benchmark circuit", seconds=time.perf_counter() - t)
    tune["tuned_entries"] = sum(1 for v in G.gkr_tune_get()[4:] if v != 0xFF)
    if args.write_tune:
        save_tune_table(G, args.write_tune, f"F2 n=2^{args.log_n}, seed {seed}")

    def step(times):
        t0 = time.perf_counter()
        m, _ = G.gkr_prove(gc, xt, seed, want_chals=False)
        t1 = time.perf_counter()
        ok = G.gkr_verify(gc, xt, seed, m)[0]
        t2 = time.perf_counter()
        fm, _ = G.f2_sumcheck_prove(at, fseed)
        t3 = time.perf_counter()
        fok = G.f2_sumcheck_verify(at, fseed, fm)[0]
        t4 = time.perf_counter()
        if not (ok and fok):
            raise SystemExit("verifier rejected an honest transcript")
        times.append((t1 - t0, t2 - t1, t3 - t2, t4 - t3))

    for _ in range(args.warmup):
        step([])
    times = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(times)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # Per-kernel timing: HIP events around every launch (on the library's
    # launch stream) cost CPU time per launch, so they run in a replay of the
    # same proofs after the timed region, leaving the timed steps clean.
    G.gkr_profile_read()
    G.gkr_profile_launches()
    G.gkr_profile_enable(2)
    for _ in range(args.steps):
        G.gkr_prove(gc, xt, seed, want_chals=False)
    G.gkr_profile_enable(0)
    prof = G.gkr_profile_read()
    per_launch = G.gkr_profile_launches()

    if args.copy_calibration_mib:
        src = torch.empty(args.copy_calibration_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    peak_mm = mulmod_rate(G, torch, dev)
    alu_peak = ALU_PEAK_MULMOD
    T = np.array(times)
    prove_s = float(T[:, 0].mean())
    value = circ.gates / prove_s
    # dominant prover kernel: the step kernel with the most device time
    prover_classes = [k for k in prof if prof[k][1] > 0 and k.startswith("step_") and k[5:] in STEP_KINDS]
    dom = max(prover_classes, key=lambda k: prof[k][0])
    ms, launches, by, mo = prof[dom]
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    alu_achieved = mo / (ms * 1e-3) if ms > 0 else 0.0
    traffic = measured_traffic(dom)
    fh, fa = achieved / HBM_PEAK_GBS, alu_achieved / alu_peak
    # both bounds per size class (ceil log2 of a launch's work items)
    buckets = {}
    for cls, sc, lms, lby, lmo in per_launch:
        if cls != dom:
            continue
        b = buckets.setdefault(sc, [0, 0.0, 0.0, 0.0])
        b[0] += 1
        b[1] += lms
        b[2] += lby
        b[3] += lmo
    by_size = []
    for sc in sorted(buckets):
        n_, t_, b_, m_ = buckets[sc]
        gbs, mps = b_ / (t_ * 1e-3) / 1e9, m_ / (t_ * 1e-3)
        by_size.append({"size_class_log2_items": sc, "launches_per_proof": n_ / args.steps,
                        "avg_launch_us": t_ * 1e3 / n_, "bytes_per_launch": b_ / n_,
                        "hbm_frac": gbs / HBM_PEAK_GBS, "alu_frac": mps / alu_peak,
                        "bound": "alu" if mps / alu_peak > gbs / HBM_PEAK_GBS else "hbm"})
    if fa > fh:
        roof = {"bound": "alu", "achieved": alu_achieved / 1e9, "peak": alu_peak / 1e9,
                "unit": "Gmulmod/s", "frac": fa}
    else:
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fh}
    roof.update({"traffic": traffic, "kernel": rocprof_kernel_name(dom), "class": dom,
                 "avg_launch_us": ms * 1e3 / launches if launches else None,
                 "algorithmic_bytes_per_launch": by / launches if launches else None,
                 "algorithmic_products_per_launch": mo / launches if launches else None,
                 "hbm_frac": fh, "alu_frac": fa, "by_size_class": by_size,
                 "alu_peak_note": "21 VALU instructions per modular product (the field module's "
                                  "compiled product), one wave64 instruction per SIMD per 4 cycles, "
                                  "256 CUs x 4 SIMDs at 2.4 GHz; measured product probe "
                                  f"{peak_mm / 1e9:.0f} Gmulmod/s"})
    line = {
        "metric": "GKR prover gates/s (batched vs plain, bit-exact); proofs/s + p50/p99 latency",
        "value": value,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"F2 GKR n=2^{args.log_n} (seed 2) prove+verify, plus F2 "
                               f"sum-check n=2^{args.f2sc_log_n} (seed 2) prove+verify; plain "
                               "path (one proof, one launch per step)",
                   "gates": circ.gates, "rounds": gc.rounds, "layers": len(circ.sizes),
                   "field": "F_p, p=2^61-1"},
        "ms_breakdown": {"gkr_prove": prove_s * 1e3, "gkr_verify": float(T[:, 1].mean()) * 1e3,
                         "f2_sumcheck_prove": float(T[:, 2].mean()) * 1e3,
                         "f2_sumcheck_verify": float(T[:, 3].mean()) * 1e3},
        "kernels_per_proof": {k: {"ms": v[0] / args.steps, "launches": v[1] / args.steps,
                                  "GB_per_s": (v[2] / (v[0] * 1e-3) / 1e9) if v[0] > 0 else None,
                                  "Gmulmod_per_s": (v[3] / (v[0] * 1e-3) / 1e9) if v[0] > 0 else None}
                              for k, v in prof.items() if v[1]},
        "autotune": tune,
        "roofline": roof,
    }
    # The line's kernels, rated by the planner's count of their modular
    # products: the sums over eq tables (step_line, one product per entry and
    # line point) and the fold of wide layers (step_lfold, ~6 an entry).
    line_k = {}
    for cls in ("step_line", "step_lfold"):
        if cls in prof and prof[cls][0] > 0 and prof[cls][3] > 0:
            rate = prof[cls][3] / (prof[cls][0] * 1e-3)
            line_k[cls] = {"mulmods_per_proof": prof[cls][3] / args.steps,
                           "launches_per_proof": prof[cls][1] / args.steps,
                           "mulmods_per_s": rate, "frac_of_peak": rate / alu_peak}
    line["alu"] = {"mulmod_peak_per_s": alu_peak, "mulmod_probe_per_s": peak_mm,
                   "peak_probe": "2^24 independent chains of 256 dependent products",
                   "line_kernels": line_k}
    note("plain leg done", f"{prove_s * 1e3:.3f} ms/proof")
    if not args.no_configs:
        note("configuration legs")
        line["configs"] = {
            "F2 n=2^10": config_leg(G, W, np, torch, W.c1_f2, "F2 GKR n=2^10, seed 1", 50),
            "MatMult N=256": config_leg(G, W, np, torch, W.c3_matmult, "MatMult GKR N=256, seed 3", 10)}
    if not args.no_configs:
        note("input-size sweep")
        line["size_sweep"] = size_sweep(G, W, np, torch)
    if not args.no_batch:
        note("batch leg")
        line["batched"] = batch_leg(G, W, np, torch, max(1, args.steps // 2), args.autotune != "off",
                                    alu_peak)
    if not args.no_serve:
        k = max(1, args.serve_points)
        rates = [0.1 * 15.0 ** (j / (k - 1)) for j in range(k)] if k > 1 else [1.0]
        note("serve leg")
        line["served"] = serve_leg(G, W, np, args.serve_requests, 200, rates, alu_peak)
    kept = {}
    if not args.no_table2:
        note("Table 2 circuits")
        line["table2_circuits"], kept = table2_leg(G, W, np, torch, 3, not args.no_cpu_baseline,
                                                   () if args.no_ooc else ("F0", "MatMult"))
    if kept:
        note("out-of-core leg")
        line["out_of_core"] = ooc_leg(G, np, torch, kept, 2)
    kept = None
    if not args.no_table3:
        note("Table 3 leg")
        line["table3_noninteractive_f2"] = table3_leg(G, np, torch, 5, not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        note("oracle on the host cores")
        cb = cpu_baseline(W, np)
        line["cpu_baseline"] = cb["headline"]
        line["cpu_oracle_samples"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
