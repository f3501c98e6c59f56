"""Builds libivde.so (gfx950 HIP kernels + C ABI host code) in-tree."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libivde.so")
SOURCES = ["kernels.hip", "terms.hip", "host.cpp", "batch.cpp", "server.cpp", "autotune.cpp", "window.cpp", "intra.cpp", "graphcut.cpp", "depth.cpp", "noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# hipcc forms packed FP32 instructions from ordinary float code; they are
# kept out of every kernel here.
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-bitwise-instead-of-logical", f"--offload-arch={ARCH}", *NO_PACKED_FP32]


# Host-code sanitizer build (libivde_san.so): AddressSanitizer and
# UndefinedBehaviorSanitizer on the host side of every source only; the GPU
# code objects are built as usual.  Load it with the ASan runtime preloaded
# and IVDE_LIB pointing at it (see sanitize_env()).
SAN_LIB = os.path.join(HERE, "libivde_san.so")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


# Measurement build (libivde_stage.so): the one-label-per-lane sweep stages
# target footprints of up to this many texels per wave in LDS.
STAGE_LIB = os.path.join(HERE, "libivde_stage.so")
STAGE_TEXELS = 624


# Measurement build (libivde_tested.so): the pixel-pair sweep tests every
# sample against the validity band, also on chunks shown to lie inside it.
TESTED_LIB = os.path.join(HERE, "libivde_tested.so")


def _compile(src: str, sanitize: bool = False, stage_texels: int = 0, tested: bool = False) -> str:
    tag = ".san" if sanitize else f".stage{stage_texels}" if stage_texels else ".tested" if tested else ""
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + tag + ".o")
    extra = [f"-DIVDE_STAGE_TEXELS={stage_texels}"] if stage_texels else ["-DIVDE_PAIR_INSIDE=0"] if tested else []
    cmd = [HIPCC, *COMMON, *(SAN_HOST if sanitize else []), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")
    return obj


def build(verbose: bool = False, sanitize: bool = False, stage_texels: int = 0, tested: bool = False) -> str:
    """Compile every source and link libivde.so next to this file; with
    sanitize, the host-sanitizer build libivde_san.so; with stage_texels,
    the LDS-staging measurement build libivde_stage.so; with tested, the
    measurement build libivde_tested.so (only kernels.hip differs: the
    objects of the other sources are the default build's)."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def one(src):
        if tested and src != "kernels.hip":
            obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
            return obj if os.path.exists(obj) else _compile(src)
        return _compile(src, sanitize, stage_texels, tested)

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(one, srcs))
    lib = SAN_LIB if sanitize else STAGE_LIB if stage_texels else TESTED_LIB if tested else LIB
    tmp = lib + ".tmp"
    link_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"] \
        if sanitize else []
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *link_san, "-o", tmp, *objs, "-lpthread"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


MIX_JSON = LIB + ".sweep_mix.json"
# the bilinear FP32-store instantiations of the two sweep forms
SWEEP_SYMBOLS = {
    "one_pixel": "_ZN4ivde12_GLOBAL__N_121k_sweep_persistent_j1ILb1ELb0ELb0EEEvPKNS_7ProblemEPKNS_4TaskEPKiPil",
    "pairs": "_ZN4ivde12_GLOBAL__N_113k_sweep_pairsILb1ELb0ELi2ELb0EEEvPKNS_7ProblemEPKNS_4TaskEPKiPil",
    "quads": "_ZN4ivde12_GLOBAL__N_113k_sweep_pairsILb1ELb0ELi4ELb0EEEvPKNS_7ProblemEPKNS_4TaskEPKiPil",
    # texels of 16-bit code values (12- to 16-bit content)
    "one_pixel16": "_ZN4ivde12_GLOBAL__N_121k_sweep_persistent_j1ILb1ELb0ELb1EEEvPKNS_7ProblemEPKNS_4TaskEPKiPil",
    "pairs16": "_ZN4ivde12_GLOBAL__N_113k_sweep_pairsILb1ELb0ELi2ELb1EEEvPKNS_7ProblemEPKNS_4TaskEPKiPil",
    "quads16": "_ZN4ivde12_GLOBAL__N_113k_sweep_pairsILb1ELb0ELi4ELb1EEEvPKNS_7ProblemEPKNS_4TaskEPKiPil",
}


def _loops(text: str, symbol: str):
    """(name, instruction mnemonics) of every block of `symbol` that ends in
    a branch back to itself."""
    import re
    start = text.index(symbol + ":")
    end = text.index(".Lfunc_end", start)
    blocks, name, body = {}, None, []
    for line in text[start:end].splitlines():
        m = re.match(r"^(\.LBB\w+):", line)
        if m or line.startswith("; %bb."):     # labelled and fall-through blocks
            if name:
                blocks[name] = body
            name, body = (m.group(1) if m else None), []
        elif name:
            ins = line.split(";")[0].strip()
            if ins and not ins.startswith("."):
                body.append(ins)
    if name:
        blocks[name] = body
    return [(n, [b.split()[0] for b in body]) for n, body in blocks.items()
            if body and body[-1].split()[0].startswith("s_cbranch") and body[-1].split()[-1] == n]


def sweep_mix(verbose: bool = False) -> dict:
    """Instruction counts of the sweep's hot loops, from the gfx950 assembly
    of the library as compiled (the bilinear FP32-store kernels; each loop's unrolled
    copy, the one with the fewest compares where the kernel has several):
    one_pixel, the one-pixel sweep's four-pixel loop for targets proven in
    front of every level point (8 gathers, one wave step per pixel); and the
    pixel-pair sweep's loops over three pairs (6 gathers, one LDS record read
    per wave step of two pixels at 32 levels): pairs_inside on projected
    records of chunks inside the validity band (no per-sample tests),
    pairs_tested on projected records with the band test, pairs_records on
    {x, y} records with the sign tests; quads_* the same loops of the
    four-pixel sweep; and each of these again, suffixed 16, for texels of
    16-bit code values (one_pixel16, pairs16_*, quads16_*).  Written next to
    the library for the benchmark's issue model."""
    import json

    with tempfile.TemporaryDirectory() as td:
        asm = os.path.join(td, "kernels.s")
        r = subprocess.run([HIPCC, *COMMON, "--cuda-device-only", "-S", "-o", asm, os.path.join(CSRC, "kernels.hip")],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"assembly of kernels.hip failed:\n{r.stderr}")
        text = open(asm).read()
    wanted = {
        "one_pixel": (SWEEP_SYMBOLS["one_pixel"], lambda ops, g: g == 8, 4),
        "pairs_inside": (SWEEP_SYMBOLS["pairs"],
                         lambda ops, g: g == 6 and "ds_read_u16" in ops and "v_med3_f32" not in ops, 3),
        "pairs_tested": (SWEEP_SYMBOLS["pairs"],
                         lambda ops, g: g == 6 and "ds_read_u16" in ops and "v_med3_f32" in ops, 3),
        "pairs_records": (SWEEP_SYMBOLS["pairs"], lambda ops, g: g == 6 and "ds_read_u16" not in ops, 3),
    }
    def side16(ops):
        """16-bit code values: projected records read FP32 Cb, Cr beside the record."""
        return "ds_read_b64" in ops or "ds_read2_b64" in ops

    # (the two-pixel kernel for them keeps two pairs in flight: 4 gathers per
    # 2 wave steps; its four-pixel kernel three, as with halves)
    for sym, pre, g_it in ((SWEEP_SYMBOLS["pairs16"], "pairs16_", 4), (SWEEP_SYMBOLS["quads16"], "quads16_", 6)):
        steps = g_it // 2                          # two gathers per wave step
        wanted[pre + "inside"] = (sym, lambda ops, g, n=g_it: g == n and side16(ops) and "v_med3_f32" not in ops,
                                  steps)
        wanted[pre + "tested"] = (sym, lambda ops, g, n=g_it: g == n and side16(ops) and "v_med3_f32" in ops, steps)
        wanted[pre + "records"] = (sym, lambda ops, g, n=g_it: g == n and not side16(ops), steps)
    wanted["one_pixel16"] = (SWEEP_SYMBOLS["one_pixel16"], lambda ops, g: g == 8, 4)
    for form in ("inside", "tested", "records"):   # four pixels per step with halves: the pair loops
        sym, pick, steps = wanted["pairs_" + form]
        wanted["quads_" + form] = (SWEEP_SYMBOLS["quads"], pick, steps)
    forms = {}
    for form, (sym, pick, steps) in wanted.items():
        cands = []
        for name, ops in _loops(text, sym):
            if pick(ops, sum(o == "buffer_load_dwordx4" for o in ops)):
                cands.append((sum(o.startswith("v_cmp") for o in ops), name, ops))
        if not cands:
            raise RuntimeError(f"{form} sweep loop not found in the assembly")
        _, name, ops = min(cands)
        counts = {}
        for o in ops:
            counts[o] = counts.get(o, 0) + 1
        forms[form] = {"kernel": sym, "loop": name, "wave_steps_per_iteration": steps,
                       "valu_instructions": sum(v for k, v in counts.items() if k.startswith("v_")),
                       "gathers": counts.get("buffer_load_dwordx4", 0), "counts": dict(sorted(counts.items()))}
    mix = {"forms": forms}
    with open(MIX_JSON, "w") as fh:
        json.dump(mix, fh, indent=1)
    if verbose:
        for form, m in forms.items():
            print(f"{form} sweep loop {m['loop']}: {m['valu_instructions']} VALU instructions, {m['gathers']} "
                  f"gathers per {m['wave_steps_per_iteration']} wave steps")
        print(f"-> {MIX_JSON}")
    return mix


CALIB_LIB = os.path.join(HERE, "libivde_calib.so")


def build_calib(verbose: bool = False) -> str:
    """libivde_calib.so: the calibration kernels behind the benchmark's
    roofline (instruction issue costs, shader clock, gather rate)."""
    os.makedirs(BUILD, exist_ok=True)
    obj = _compile("calib.hip")
    tmp = CALIB_LIB + ".tmp"
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, obj], capture_output=True,
                       text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, CALIB_LIB)
    if verbose:
        print(f"built {CALIB_LIB}")
    return CALIB_LIB


def sanitize_env() -> dict:
    """Environment that runs Python against libivde_san.so: the ASan runtime
    preloaded (the interpreter itself is not instrumented), leaks not
    reported (the interpreter's own allocations would be), any report
    fatal."""
    import glob
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        raise RuntimeError("no ASan runtime found under /opt/rocm/llvm")
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt[-1], IVDE_LIB=SAN_LIB, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return env


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv,
          stage_texels=STAGE_TEXELS if "--stage" in sys.argv else 0)
