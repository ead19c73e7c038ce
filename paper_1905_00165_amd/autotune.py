"""Autotuner of the launch-sequence constants (csrc/tuning.h), run on the GPU.

The library reads its panel widths, size-group widths and small-problem
cutover from csrc/tuning.h at build time. This script measures candidate
values on the GPU and rewrites that file with the fastest ones, recording the
measurements in its comment block. Every constant is a function of (storage,
precision, problem size) only, so tuning never makes a result depend on the
rest of a batch; the panel widths do change the blocking, hence the rounding
of a sample, which is why they are chosen here once per build and not per
call.

Each candidate is a copy of csrc/ with its own tuning.h: only api.hip (the
host side, which holds these constants) is recompiled and linked with the
kernel objects of the regular build (paper_1905_00165_amd/_build), and a
fresh process times it through the binding (so every candidate loads its own
library). Workloads:

  - small-problem cutover: batches of 1024 Hermitian kernels of one size n in
    {32, 64, ..., 192} (FP32 storage, the L-ensemble construction), with the
    small path everywhere against the blocked path everywhere, per precision;
    the cutover is the largest n below which the small path is faster at
    every measured size;
  - size groups: the 4096-kernel L-ensemble batch (n ~ U{64..1024}, FP32),
    narrow widths 64 / 128 / 256, split and FP64;
  - panel widths: LDL^H on the projection kernel n = 16384 (8 samples), split
    (six products) 2048 / 4096 and FP64 1024 / 2048 / 4096; LU on the similarity
    kernel n = 8192 (8 samples), 256 / 512 / 1024.

Usage (on an MI355X, after a regular build):
    python -m paper_1905_00165_amd.autotune [--write] [--quick]
Without --write the chosen values are printed only.
"""
import argparse
import json
import os
import re
import shutil
import subprocess
import sys
import tempfile
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
TUNING = os.path.join(CSRC, "tuning.h")

DEFAULTS = {"kB0LdlhSplit": 4096, "kB0LdlhFp64": 4096, "kB0Lu": 2048, "kGroupNarrow": 128,
            "kGroupSplitN": 2048, "kGroupWide": 1024, "kSmallCutover": [128, 128, 128, 128]}


def read_tuning(path=TUNING):
    text = open(path).read()
    vals = {}
    for k, v in DEFAULTS.items():
        if isinstance(v, list):
            m = re.search(k + r"\[4\] = \{([^}]*)\}", text)
            vals[k] = [int(x) for x in m.group(1).split(",")]
        else:
            m = re.search(r"\b" + k + r" = (\d+);", text)
            vals[k] = int(m.group(1))
    return vals


def render(vals, record):
    """tuning.h with the given values and the measurement record."""
    out = open(TUNING).read()
    for k, v in vals.items():
        if isinstance(v, list):
            out = re.sub(k + r"\[4\] = \{[^}]*\}", k + "[4] = {" + ", ".join(str(x) for x in v) + "}", out)
        else:
            out = re.sub(r"(\b" + k + r" = )\d+;", r"\g<1>" + str(v) + ";", out)
    body = out.split("#pragma once", 1)[1]
    head = ("// Tuned constants of the launch sequence, each a function of (storage,\n"
            "// precision, problem size) only, so that a result never depends on the rest\n"
            "// of its batch. paper_1905_00165_amd/autotune.py measures the candidates on\n"
            "// the GPU and writes this file; its record of the measurements is the comment\n"
            "// block below.\n")
    rec = "".join("// " + line + "\n" for line in record)
    return head + rec + "#pragma once" + body


def build_variant(vals, workdir):
    """libdpp.so with `vals` in tuning.h: api.hip recompiled, kernels reused."""
    from . import build as B
    src = os.path.join(workdir, "csrc")
    shutil.copytree(CSRC, src)
    text = open(os.path.join(src, "tuning.h")).read()
    for k, v in vals.items():
        if isinstance(v, list):
            text = re.sub(k + r"\[4\] = \{[^}]*\}", k + "[4] = {" + ", ".join(str(x) for x in v) + "}", text)
        else:
            text = re.sub(r"(\b" + k + r" = )\d+;", r"\g<1>" + str(v) + ";", text)
    open(os.path.join(src, "tuning.h"), "w").write(text)
    flags = [f if f != CSRC else src for f in B.FLAGS]
    api_o = os.path.join(workdir, "api.hip.o")
    subprocess.run([B.HIPCC, *flags, "-c", os.path.join(src, "api.hip"), "-o", api_o], check=True,
                   capture_output=True)
    objs = [os.path.join(OBJ, f) for f in sorted(os.listdir(OBJ))
            if f.endswith(".hip.o") and f != "api.hip.o"]
    lib = os.path.join(workdir, "libdpp.so")
    subprocess.run([B.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", api_o, *objs, "-o", lib],
                   check=True, capture_output=True)
    return lib


# ------------------------------------------------------------ timing workers
# Each runs in its own process with the candidate library, prints one JSON line.

def _worker(lib, task, arg):
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    from paper_1905_00165_amd import binding as B
    from paper_1905_00165_amd import workloads as W
    B.LIB_PATH = lib
    dev = torch.device("cuda:0")

    def timed(step, reps):
        step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            step()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def graph_timed(step, reps):
        """ms per replay of one captured call (the host cost of marshalling
        a large batch stays out of the measurement)."""
        step()
        torch.cuda.synchronize()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        ms = timed(g.replay, reps)
        del g
        return ms

    res = {}
    if task == "small":
        n, count = int(arg), 1024
        Ks = [W.lensemble_kernel(n, seed=900000 + i, out=torch.empty((n, n), dtype=torch.float32,
                                                                     device=dev).t())
              for i in range(count)]
        us = [torch.from_numpy(W.uniform_stream(n, seed=90000 + i)).to(dev) for i in range(count)]
        As = [torch.empty_like(K) for K in Ks]
        for prec in (0, 1, 2, 3):
            ws = torch.empty(B.dpp_workspace_size_batched(True, B.DPP_F32, [n] * count, prec),
                             dtype=torch.uint8, device=dev)
            res[prec] = graph_timed(lambda: B.dpp_sample_ldlh_batched(As, us, prec=prec, ws=ws, Ks=Ks), 10)
    elif task == "groups":
        count = 4096
        ns = W.lensemble_batch_sizes(count, seed=4)
        Ks = [W.lensemble_kernel(int(n), seed=400000 + i,
                                 out=torch.empty((int(n), int(n)), dtype=torch.float32, device=dev).t())
              for i, n in enumerate(ns)]
        us = [torch.from_numpy(W.uniform_stream(int(n), seed=4000 + i)).to(dev) for i, n in enumerate(ns)]
        As = [torch.empty_like(K) for K in Ks]
        for prec in (0, 2):
            ws = torch.empty(B.dpp_workspace_size_batched(True, B.DPP_F32, [int(x) for x in ns], prec),
                             dtype=torch.uint8, device=dev)
            res[prec] = graph_timed(lambda: B.dpp_sample_ldlh_batched(As, us, prec=prec, ws=ws, Ks=Ks), 3)
            del ws
    elif task in ("b0_ldlh_split", "b0_ldlh_fp64"):
        n, r, bsz = 16384, 4096, 8
        prec = 2 if task == "b0_ldlh_split" else 0
        K = W.projection_kernel(n, r, seed=2, device=dev)
        us = [torch.from_numpy(W.uniform_stream(n, seed=2000 + i)).to(dev) for i in range(bsz)]
        As = [torch.empty_like(K) for _ in range(bsz)]
        ws = torch.empty(B.dpp_workspace_size_batched(True, B.DPP_F64, [n] * bsz, prec),
                         dtype=torch.uint8, device=dev)
        res[prec] = timed(lambda: B.dpp_sample_ldlh_batched([A.t() for A in As], us, prec=prec, ws=ws,
                                                            Ks=[K.t()] * bsz), 2)
    elif task == "b0_lu":
        n, bsz = 8192, 8
        K, _ = W.similarity_kernel(n, seed=3, device=dev)
        us = [torch.from_numpy(W.uniform_stream(n, seed=3000 + i)).to(dev) for i in range(bsz)]
        As = [torch.empty_like(K) for _ in range(bsz)]
        for prec in (0, 2):
            ws = torch.empty(B.dpp_workspace_size_batched(False, B.DPP_F64, [n] * bsz, prec),
                             dtype=torch.uint8, device=dev)
            res[prec] = timed(lambda: B.dpp_sample_lu_batched(As, us, prec=prec, ws=ws, Ks=[K] * bsz), 2)
    print(json.dumps({"task": task, "arg": arg, "ms": res}), flush=True)


_LIBS = {}
_TMP = None


def variant_lib(vals):
    """The candidate library for `vals`, built once per distinct set."""
    global _TMP
    key = json.dumps(vals, sort_keys=True)
    if key not in _LIBS:
        if _TMP is None:
            _TMP = tempfile.TemporaryDirectory(prefix="dpp_tune_")
        d = os.path.join(_TMP.name, str(len(_LIBS)))
        os.makedirs(d)
        _LIBS[key] = build_variant(vals, d)
    return _LIBS[key]


def measure(vals, task, arg, log):
    lib = variant_lib(vals)
    t0 = time.time()
    r = subprocess.run([sys.executable, "-m", "paper_1905_00165_amd.autotune", "--worker", lib,
                        task, str(arg)], cwd=ROOT, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError(f"worker {task} {arg} failed:\n{r.stderr[-2000:]}")
    out = json.loads(r.stdout.strip().splitlines()[-1])
    ms = {int(k): round(v, 4) for k, v in out["ms"].items()}
    shown = {k: vals[k] for k in ("kSmallCutover", "kGroupNarrow", "kB0LdlhSplit", "kB0LdlhFp64",
                                  "kB0Lu")}
    log(f"[autotune] {task} arg={arg} {shown} -> {ms} ({time.time() - t0:.0f} s)")
    return ms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--worker", nargs=3, metavar=("LIB", "TASK", "ARG"))
    ap.add_argument("--write", action="store_true", help="rewrite csrc/tuning.h with the choice")
    ap.add_argument("--quick", action="store_true", help="small-problem cutover only")
    a = ap.parse_args()
    if a.worker:
        _worker(a.worker[0], a.worker[1], a.worker[2])
        return

    def log(msg):
        print(msg, flush=True)

    if not os.path.isdir(OBJ) or not any(f.endswith(".hip.o") for f in os.listdir(OBJ)):
        from . import build as B
        log("[autotune] building the kernel objects")
        B.build()
    base = read_tuning()
    record = [f"Record of the autotune run of {time.strftime('%Y-%m-%d')} (ms per call, by precision 0 = FP64,",
              "1 = split x3, 2 = split x6, 3 = FP16 split):"]
    chosen = dict(base)

    # Small-problem cutover: small path everywhere against blocked everywhere.
    sizes = [32, 64, 96, 128, 160, 192]
    small_on = dict(base, kSmallCutover=[192, 192, 192, 192])
    small_off = dict(base, kSmallCutover=[0, 0, 0, 0])
    cut = [0, 0, 0, 0]
    faster = [True, True, True, True]
    for n in sizes:
        on = measure(small_on, "small", n, log)
        off = measure(small_off, "small", n, log)
        record.append(f"  1024 kernels of n = {n}: small path {on}, blocked {off}")
        for p in (0, 1, 2, 3):
            faster[p] = faster[p] and on[p] < off[p]
            if faster[p]:
                cut[p] = n
    chosen["kSmallCutover"] = cut
    record.append(f"  -> kSmallCutover = {cut}")

    if not a.quick:
        best = None
        for w in (64, 128, 256):
            v = dict(chosen, kGroupNarrow=w)
            ms = measure(v, "groups", 0, log)
            record.append(f"  4096 L-ensembles, group width {w}: {ms}")
            score = ms[0] + ms[2]
            if best is None or score < best[0]:
                best = (score, w)
        chosen["kGroupNarrow"] = best[1]
        record.append(f"  -> kGroupNarrow = {best[1]}")
        for key, task, cands, prec in (("kB0LdlhSplit", "b0_ldlh_split", (2048, 4096), 2),
                                       ("kB0LdlhFp64", "b0_ldlh_fp64", (1024, 2048, 4096), 0),
                                       ("kB0Lu", "b0_lu", (512, 1024, 2048, 4096), None)):
            best = None
            for c in cands:
                ms = measure(dict(chosen, **{key: c}), task, 0, log)
                record.append(f"  {task} {key} = {c}: {ms}")
                score = sum(ms.values()) if prec is None else ms[prec]
                if best is None or score < best[0]:
                    best = (score, c)
            chosen[key] = best[1]
            record.append(f"  -> {key} = {best[1]}")

    log("[autotune] chosen: " + json.dumps(chosen))
    if a.write:
        text = render(chosen, record)  # reads the current file: before it is truncated
        with open(TUNING, "w") as f:
            f.write(text)
        log(f"[autotune] wrote {TUNING}")
    else:
        log("\n".join(record))


if __name__ == "__main__":
    main()
