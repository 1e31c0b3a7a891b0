"""Build ``libpid.so`` (the C-ABI library) for gfx950 with hipcc, in-tree.

Usage: ``python -m paper_2512_15187_amd.build`` (or ``build()`` from Python).
Every call recompiles all sources.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpid.so")
# stand-alone counter-run driver (no torch), linked against libpid.so
MEASURE = os.path.join(HERE, "pid_measure")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of the device code on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
REPORT = os.path.join(OUT_DIR, "resource_usage.txt")
SOURCES = ["k_gram_f32.hip", "k_gram_models.hip", "k_gram_f16.hip", "k_gram_f64u8.hip", "k_pidmean.hip", "k_gram.hip", "k_misc.hip", "k_bands.hip", "k_bits.hip", "static_scratch.hip", "api.cpp", "plan.cpp", "server.cpp", "timing.cpp"]


def _compile(src: str):
    obj = os.path.join(OUT_DIR, os.path.basename(src) + ".o")
    lang = [] if src.endswith(".hip") else ["-x", "hip"]
    # kernel sources keep their device assembly (checked below) and report
    # register use
    extra = ["-Rpass-analysis=kernel-resource-usage", "-save-temps"] if src.endswith(".hip") else []
    tmp = os.path.join(OUT_DIR, "tmp_" + os.path.basename(src))
    os.makedirs(tmp, exist_ok=True)
    cmd = [HIPCC, *COMMON, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=tmp)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if src.endswith(".hip"):
        for f in os.listdir(tmp):
            if f.endswith(f"-{ARCH}.s"):
                check_m0(os.path.join(tmp, f))
    shutil.rmtree(tmp, ignore_errors=True)
    return obj, r.stderr


def check_m0(asm_path: str):
    """The loads into LDS are written as inline assembly that sets M0 itself.
    Fail if the compiled device code uses M0 anywhere else: the compiler
    could then hold a value in M0 across such a load."""
    lines = [l.strip() for l in open(asm_path) if l.strip() and not l.strip().startswith(";")]
    bad = []
    for i, l in enumerate(lines):
        if re.search(r"\bm0\b", l):
            ok = (l.startswith("s_mov_b32 m0, ") and i + 1 < len(lines)
                  and re.match(r"buffer_load_dword\w* v\d+, s\[\d+:\d+\], (0|s\d+) offen lds$", lines[i + 1]))
            if not ok:
                bad.append(l)
    if bad:
        raise RuntimeError(f"{os.path.basename(asm_path)}: M0 used outside the LDS loads: {bad[:5]}")


def resource_report(remarks: str):
    """(kernel, vgprs, scratch bytes per lane) from -Rpass-analysis remarks."""
    out = []
    # (the remark prefix differs with -save-temps: "file:l:c: remark: Function
    # Name:" or "remark: file:l:c: Function Name:")
    for block in re.split(r"Function Name: ", remarks)[1:]:
        name = block.split()[0]
        v = re.search(r"VGPRs: (\d+)", block)
        sc = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", block)
        out.append((name, int(v.group(1)) if v else -1, int(sc.group(1)) if sc else 0))
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in results]
    report = [r for _, rem in results for r in resource_report(rem)]
    if not report:
        raise RuntimeError("no kernel resource remarks were parsed")
    with open(REPORT, "w") as fh:
        for name, vgpr, scratch in report:
            fh.write(f"{name}\tvgpr={vgpr}\tscratch={scratch}\n")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    shutil.move(tmp, LIB)
    cmd = [HIPCC, *COMMON, os.path.join(CSRC, "measure_main.hip"), "-o", MEASURE + ".tmp", "-L" + HERE, "-lpid",
           "-Wl,-rpath,$ORIGIN"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"driver build failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    shutil.move(MEASURE + ".tmp", MEASURE)
    if verbose:
        print(f"built {LIB} and {MEASURE}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
