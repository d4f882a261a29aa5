"""Builds libldpc.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Each translation unit is compiled to its own object in parallel; the decode
kernels are compiled once per (block rows, max degree) shape. Flags:
-ffp-contract=off keeps every FP32 product and sum separately rounded (the
decoder must match an IEEE evaluation of its definition bit for bit), and
packed FP32 instructions are disabled.
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libldpc.so")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("LDPC_OFFLOAD_ARCH", "gfx950")
# (block rows, max check degree) shapes of the decode kernels; must match
# the table in csrc/decode_dispatch.cpp.
SHAPES = [(4, 20), (6, 20), (8, 16), (12, 12), (12, 16), (16, 26)]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function"]
GPU = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


JIT_SOURCES = [("jit_decode.hip", "kJitDecodeSource"), ("jit_nms.hip", "kJitNmsSource"),
               ("jit_batch.hip", "kJitBatchSource"), ("jit_flood.hip", "kJitFloodSource"),
               ("jit_q16.hip", "kJitQ16Source"), ("jit_h2.hip", "kJitH2Source")]


def _embed_jit_source():
    """Writes _build/jit_source.cpp: the hipRTC kernel sources as C++ strings."""
    delim = "LDPCJIT"
    out = os.path.join(OBJ, "jit_source.cpp")
    parts = ["// generated from csrc/jit_*.hip by build.py", "namespace ldpc {"]
    for fname, sym in JIT_SOURCES:
        with open(os.path.join(CSRC, fname)) as fh:
            text = fh.read()
        assert ")" + delim not in text
        parts.append(f"extern const char {sym}[];")
        parts.append(f"const char {sym}[] = R\"{delim}(\n{text}){delim}\";")
    parts.append("}")
    with open(out, "w") as fh:
        fh.write("\n".join(parts) + "\n")
    return out


def _units():
    units = [("ldpc_capi.cpp", [], "ldpc_capi.o"),
             ("jit.cpp", [], "jit.o"),
             ("tune.cpp", [], "tune.o"),
             ("batch.cpp", [], "batch.o"),
             (os.path.join(OBJ, "jit_source.cpp"), [], "jit_source.o"),
             ("decode_dispatch.cpp", [], "decode_dispatch.o"),
             ("frame_kernels.hip", [], "frame_kernels.o"),
             ("batch_scratch.hip", [], "batch_scratch.o")]
    for kind in ("f32", "i8"):
        for mb, d in SHAPES:
            units.append((f"decode_{kind}.hip", [f"-DLDPC_MB={mb}", f"-DLDPC_D={d}"],
                          f"decode_{kind}_{mb}_{d}.o"))
    return units


def _compile(unit, verbose):
    src, defs, obj = unit
    out = os.path.join(OBJ, obj)
    cmd = ["hipcc", "-c"] + GPU + COMMON + defs + ["-o", out, os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    msg = "\n".join(l for l in (res.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    return out, res.returncode, msg


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(OBJ, exist_ok=True)
    _embed_jit_source()
    jobs = jobs or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda u: _compile(u, verbose), _units()))
    errors = [(o, rc, m) for o, rc, m in results if rc != 0]
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(f"{o}: {m}" for o, rc, m in errors))
    for o, rc, m in results:
        if verbose and m.strip():
            print(m)
    tmp = LIB + ".tmp"
    link = (["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + [o for o, _, _ in results]
            + ["-lhiprtc"])
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=False))
