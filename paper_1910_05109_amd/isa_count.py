"""Instruction count of the kernels' steady-state loops on gfx950.

The paper counts the SIMD instructions its AVX-512 loops spend per 512-bit
register, leaving out loads and stores: 3 per 48 input bytes to encode and 5
per 64 characters to decode (Sections "Encoding" and "Decoding").  This tool
compiles the library for gfx950, finds the software-pipelined main loop of
k_encode, k_decode and k_validate in the generated assembly (the loop that
handles two rounds of U lane chunks per iteration), and counts its
instructions by kind.  Dividing by the bytes one wave handles per iteration
gives wave instructions per input byte, the GPU analogue of the paper's
figure: one wave instruction acts on 64 lanes as one AVX-512 instruction acts
on 64 bytes.

  python -m paper_1910_05109_amd.isa_count
"""
from __future__ import annotations

import os
import re
import subprocess
import tempfile

from .build import CSRC, FLAGS, hipcc

# kernel template instance -> (mangled-name fragment, unroll U, input bytes per
# lane chunk); the loop body holds two rounds of U chunks
KERNELS = {
    "k_encode<4, nt>": ("k_encodeILi4ELb1E", 4, 12),
    "k_decode<8, nt>": ("k_decodeILi8ELb1E", 8, 16),
    "k_validate<8, nt>": ("k_validateILi8ELb1E", 8, 16),
}
KINDS = (("vmem load", r"^(global|buffer)_load"), ("vmem store", r"^(global|buffer)_store"),
         ("lds", r"^ds_"), ("valu", r"^v_"), ("salu", r"^s_(?!waitcnt|cbranch|branch|nop)"),
         ("wait/branch", r"^s_(waitcnt|cbranch|branch|nop)"))


def assemble(src: str, workdir: str) -> str:
    out = os.path.join(workdir, "k.o")
    cmd = [hipcc(), *[f for f in FLAGS if f not in ("-shared", "-fPIC")], "-c", src, "-o", out,
           "--save-temps"]
    subprocess.check_call(cmd, cwd=workdir, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    base = os.path.splitext(os.path.basename(src))[0]
    with open(os.path.join(workdir, f"{base}-hip-amdgcn-amd-amdhsa-gfx950.s")) as f:
        return f.read()


def scratch_sizes(threads: int = 4) -> dict:
    """Scratch memory per lane of every kernel in the library's sources,
    {mangled kernel name: bytes}, from the device assembly's kernel
    descriptors (.amdhsa_private_segment_fixed_size).  Scratch is where the
    compiler puts what does not fit in registers or is indexed dynamically;
    every access to it is a round trip to memory."""
    from concurrent.futures import ThreadPoolExecutor
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    flags = [f for f in FLAGS if f not in ("-shared", "-fPIC")]

    def one(src: str, wd: str) -> str:
        out = os.path.join(wd, src + ".s")
        subprocess.check_call([hipcc(), *flags, "--offload-device-only", "-S",
                               os.path.join(CSRC, src), "-o", out],
                              cwd=wd, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        with open(out) as f:
            return f.read()

    sizes = {}
    with tempfile.TemporaryDirectory() as wd, ThreadPoolExecutor(threads) as pool:
        for asm in pool.map(lambda s: one(s, wd), srcs):
            for m in re.finditer(r"^\s*\.amdhsa_kernel (\S+)(.*?)^\s*\.end_amdhsa_kernel", asm,
                                 flags=re.M | re.S):
                fixed = re.search(r"\.amdhsa_private_segment_fixed_size (\d+)", m.group(2))
                sizes[m.group(1)] = int(fixed.group(1)) if fixed else 0
    return sizes


def kernel_body(asm: str, fragment: str) -> list[str]:
    m = re.search(r"^(_Z\S*" + re.escape(fragment) + r"\S*):[^\n]*$", asm, flags=re.M)
    if not m:
        raise KeyError(fragment)
    end = asm.index("s_endpgm", m.end())
    return asm[m.end(): end].split("\n")


def main_loop(lines: list[str]) -> list[str]:
    """Instructions of the loop with the most vector memory operations."""
    best: list[str] = []
    for i, ln in enumerate(lines):
        lab = re.match(r"^(\.LBB\w+):", ln)
        # the loop-header note sits on the label's line or the one after it
        if not lab or "Loop Header" not in ln + (lines[i + 1] if i + 1 < len(lines) else ""):
            continue
        label = lab.group(1)
        for j in range(i + 1, len(lines)):
            if re.search(r"s_cbranch_\w+\s+" + re.escape(label) + r"\b", lines[j]):
                body = [l.strip() for l in lines[i + 1: j + 1]]
                body = [l for l in body if l and not l.startswith((";", "."))]
                nmem = sum(1 for l in body if re.match(r"(global|buffer)_(load|store)", l))
                if nmem > sum(1 for l in best if re.match(r"(global|buffer)_(load|store)", l)):
                    best = body
                break
    return best


def count(body: list[str]) -> dict:
    c = {k: 0 for k, _ in KINDS}
    for ln in body:
        op = ln.split()[0]
        for k, pat in KINDS:
            if re.match(pat, op):
                c[k] += 1
                break
    c["total"] = len(body)
    return c


def report() -> list[dict]:
    rows = []
    with tempfile.TemporaryDirectory() as wd:
        asm = {}
        for name, (frag, u, chunk) in KERNELS.items():
            src = "b64_validate.hip" if "validate" in name else "b64_single.hip"
            if src not in asm:
                asm[src] = assemble(os.path.join(CSRC, src), wd)
            body = main_loop(kernel_body(asm[src], frag))
            c = count(body)
            lane_bytes = 2 * u * chunk            # two rounds of U chunks per iteration
            wave_bytes = 64 * lane_bytes
            compute = c["valu"] + c["lds"] + c["salu"]
            rows.append({"kernel": name, **c, "chunks_per_lane": 2 * u,
                         "input_bytes_per_wave_iteration": wave_bytes,
                         "valu_per_chunk": round(c["valu"] / (2 * u), 2),
                         "compute_instr_per_64B": round(compute * 64 / wave_bytes, 3),
                         "all_instr_per_64B": round(c["total"] * 64 / wave_bytes, 3)})
    return rows


def main():
    print(f"{'kernel':20s} {'total':>6s} {'valu':>5s} {'lds':>4s} {'salu':>5s} {'ld':>3s} {'st':>3s} "
          f"{'wait/br':>7s} {'bytes':>6s} {'valu/chunk':>10s} {'compute/64B':>11s} {'all/64B':>8s}")
    for r in report():
        print(f"{r['kernel']:20s} {r['total']:6d} {r['valu']:5d} {r['lds']:4d} {r['salu']:5d} "
              f"{r['vmem load']:3d} {r['vmem store']:3d} {r['wait/branch']:7d} "
              f"{r['input_bytes_per_wave_iteration']:6d} {r['valu_per_chunk']:10.2f} "
              f"{r['compute_instr_per_64B']:11.3f} {r['all_instr_per_64B']:8.3f}")


if __name__ == "__main__":
    main()
