"""Build the SparkCL hot-path library for gfx950.

Produces, next to this file:
  libsparkcl.so       -- the C-ABI library (HIP kernels + host runtime), built
                         with hipcc --offload-arch=gfx950;
  libsparkcl_host.so  -- the pure host logic (arena, admission, tuning cache)
                         behind a small C shim, built with g++, for CPU tests;
  libsparkcl_loadgen.so -- an open-loop serving load generator over the public
                         C ABI (submit / poll at scheduled arrival times), for
                         the serving benchmark;
  libsparkcl_probe.so -- the bench's measurement probes: a plain read-only
                         streaming kernel (the measured HBM read ceiling) and
                         register-only VALU loops (the Monte-Carlo loop's
                         measured issue ceiling);
  probe_isa.json      -- VALU instructions per loop iteration of each VALU
                         probe, read from the probe library's own assembly;
  isa.json            -- resource figures of the kernels' own gfx950 code
                         (registers, private segment, VALU instructions per
                         Philox block), read from the device assembly of this
                         same build: the no-spill guard test and the
                         Monte-Carlo ALU roofline use them.

Every HIP translation unit is compiled with -ffp-contract=off (the maps are
the binary32 definition step by step) and with packed-FP32 instructions
disabled.  Run: python -m paper_1505_01120_amd.build
"""
from __future__ import annotations

import hashlib
import json
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsparkcl.so")
HOST_LIB = os.path.join(HERE, "libsparkcl_host.so")
LOADGEN_LIB = os.path.join(HERE, "libsparkcl_loadgen.so")
PROBE_LIB = os.path.join(HERE, "libsparkcl_probe.so")
PROBE_ISA_JSON = os.path.join(HERE, "probe_isa.json")
ISA_JSON = os.path.join(HERE, "isa.json")
KERNELS = ("k_task", "k_batch", "k_serve", "k_map", "k_chain", "k_tree", "k_tree_wide", "k_wordcount",
           "k_wc_merge", "k_wc_compact", "k_wl_scan", "k_batch_mc")
ARCH = "gfx950"

HIP_SOURCES = ["kernels.hip", "noalloc.hip", "api.cpp", "arrays.cpp", "chain.cpp", "wordcount.cpp", "serve.cpp",
               "autotune.cpp", "tuning.cpp"]
HOST_SOURCES = ["tuning.cpp", "hostlogic_capi.cpp"]

COMMON = ["-std=c++17", "-O3", "-fPIC", "-fvisibility=hidden", "-Wall", "-Wextra", "-Wno-unused-parameter",
          "-I", INCLUDE, "-I", CSRC]
HIP_FLAGS = ["--offload-arch=" + ARCH, "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found: the SparkCL library needs ROCm to build")
    return p


def _run(cmd: list[str]) -> None:
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + os.path.basename(cmd[-1]))


def isa_report(asm: str) -> dict:
    """Per-kernel resources from the AMDGPU metadata, and the VALU count of
    the Philox loop (the basic block of k_batch holding the most three-way
    xors) from the device assembly text."""
    out = {}
    meta = asm[asm.find("amdhsa.kernels:"):]
    for k in KERNELS:
        # a template kernel has one entry per instantiation: keep the worst
        blocks = re.findall(r"\.name:\s+_ZN7sparkcl12_GLOBAL__N_1\d+" + k + r"[EI].*?(?=\n  - \.|\Z)",
                            meta, re.S)
        if not blocks:
            continue

        def field(name):
            vals = [re.search(r"\." + name + r":\s+(\d+)", b) for b in blocks]
            vals = [int(f.group(1)) for f in vals if f]
            return max(vals) if vals else None
        out[k] = {"vgpr": field("vgpr_count"), "sgpr": field("sgpr_count"),
                  "private_segment_bytes": field("private_segment_fixed_size"),
                  "vgpr_spills": field("vgpr_spill_count"),
                  "sgpr_spills": field("sgpr_spill_count")}
    body = re.search(r"^_ZN7sparkcl12_GLOBAL__N_17k_batch\S*:(.*?)\.end_amdhsa_kernel",
                     asm, re.S | re.M)
    if body:
        best, cur, cur_xor, best_xor = None, [], 0, 0
        for line in body.group(1).splitlines() + [".LBB_end:"]:
            t = line.strip()
            if re.match(r"^\.LBB\d+_\d+:", t) or t.startswith("; %bb."):
                if cur_xor > best_xor:
                    best, best_xor = cur, cur_xor
                cur, cur_xor = [], 0
                continue
            if not t or t.startswith(";") or t.startswith("."):
                continue
            op = t.split()[0]
            cur.append(op)
            if op == "v_bitop3_b32":
                cur_xor += 1
        if best:
            out["philox_loop"] = {"valu": sum(1 for o in best if o.startswith("v_")),
                                  "xor3": best_xor,
                                  "mad_u64_u32": best.count("v_mad_u64_u32")}
    return out


def probe_isa_report(asm: str) -> dict:
    """VALU instructions per loop iteration of each k_valu<mix> probe kernel:
    the v_ instructions of the kernel's loop block (the basic block that
    branches back to its own label)."""
    out = {}
    for m in re.finditer(r"^(_ZN12_GLOBAL__N_16k_valuILj(\d+)EEEv\S*):(.*?)\.end_amdhsa_kernel",
                         asm, re.S | re.M):
        mix, body = m.group(2), m.group(3)
        label, cur = None, []
        for line in body.splitlines():
            t = line.strip()
            lm = re.match(r"^(\.LBB\d+_\d+):", t)
            if lm:
                label, cur = lm.group(1), []
                continue
            if not t or t.startswith(";") or t.startswith("."):
                continue
            op = t.split()[0]
            cur.append(op)
            if op.startswith("s_cbranch") and label and t.split()[-1] == label:
                out[mix] = sum(1 for o in cur if o.startswith("v_"))
    return {"valu_per_iteration": out}


def build(verbose: bool = False) -> str:
    """Compile every source and link both libraries (always rebuilds)."""
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    cc = hipcc()

    def compile_hip(src: str) -> str:
        obj = os.path.join(out_dir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _run([cc, *COMMON, *HIP_FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    def device_asm() -> str:
        asm = os.path.join(out_dir, "kernels.s")
        _run([cc, *COMMON, *HIP_FLAGS, "-x", "hip", "--cuda-device-only", "-S",
              os.path.join(CSRC, "kernels.hip"), "-o", asm])
        return asm

    def probe_lib() -> None:
        # the measurement probes: a library of their own, outside the API,
        # and the VALU count of each VALU probe's loop from its assembly
        tmp = PROBE_LIB + ".tmp"
        _run([cc, *COMMON, *HIP_FLAGS, "-shared", "-x", "hip", os.path.join(CSRC, "probe.hip"),
              "-o", tmp])
        os.replace(tmp, PROBE_LIB)
        pasm = os.path.join(out_dir, "probe.s")
        _run([cc, *COMMON, *HIP_FLAGS, "-x", "hip", "--cuda-device-only", "-S",
              os.path.join(CSRC, "probe.hip"), "-o", pasm])
        with open(pasm) as f:
            rep = probe_isa_report(f.read())
        with open(PROBE_ISA_JSON + ".tmp", "w") as f:
            json.dump(rep, f, indent=1)
        os.replace(PROBE_ISA_JSON + ".tmp", PROBE_ISA_JSON)

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        asm_job = ex.submit(device_asm)
        probe_job = ex.submit(probe_lib)
        objs = list(ex.map(compile_hip, HIP_SOURCES))
        asm = asm_job.result()
        probe_job.result()
    tmp = LIB + ".tmp"
    _run([cc, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp, "-lpthread"])
    os.replace(tmp, LIB)

    tmp = HOST_LIB + ".tmp"
    _run(["g++", *COMMON, "-shared", *[os.path.join(CSRC, s) for s in HOST_SOURCES],
          "-o", tmp])
    os.replace(tmp, HOST_LIB)

    # the serving load generator: host code on top of the public C ABI
    tmp = LOADGEN_LIB + ".tmp"
    _run(["g++", *COMMON, "-shared", os.path.join(CSRC, "loadgen.cpp"), "-L", HERE,
          "-l:libsparkcl.so", "-Wl,-rpath,$ORIGIN", "-o", tmp])
    os.replace(tmp, LOADGEN_LIB)
    with open(asm) as f:
        report = isa_report(f.read())
    with open(os.path.join(CSRC, "kernels.hip"), "rb") as f:
        report["kernels_sha256_16"] = hashlib.sha256(f.read()).hexdigest()[:16]
    with open(ISA_JSON + ".tmp", "w") as f:
        json.dump(report, f, indent=1)
    os.replace(ISA_JSON + ".tmp", ISA_JSON)
    if verbose:
        print("built", LIB, "and", HOST_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
