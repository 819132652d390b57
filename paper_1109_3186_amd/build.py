"""Compile the HIP library libddx.so in-tree for gfx950."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", f) for f in ("ddx.hip", "cnn.hip", "chirp.hip", "image.hip", "incoherent.hip", "chimg.hip")]
LIB = os.path.join(HERE, "libddx.so")

# Packed-FP32 VALU instructions are kept out of the generated code.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
                                   "-o", LIB + ".tmp"] + SRC
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops' is not a recognized feature"
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if noise not in ln]
    if r.returncode != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError("hipcc failed (%d): %s" % (r.returncode, " ".join(cmd)))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(LIB + ".tmp", LIB)
    return LIB


# Host-side sanitizers: AddressSanitizer and UndefinedBehaviorSanitizer on the
# host code only (each -fsanitize behind -Xarch_host; the device code is built
# as usual, unoptimised beyond -O1).  The library is loaded by a Python that is
# not instrumented, so the ASan runtime must be preloaded (sanitizer_runtime()).
SANITIZE_FLAGS = [
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
]


def sanitizer_runtime():
    """Path of the clang ASan runtime shipped with ROCm's LLVM (to LD_PRELOAD)."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("no libclang_rt.asan-x86_64.so under /opt/rocm/lib/llvm")
    return hits[-1]


def build_sanitized(out_dir=None):
    """Build an ASan + UBSan instrumented copy of libddx.so (host code) in out_dir
    (default _build/host_sanitized at the repository root); returns its path.
    The six sources compile in parallel, then link."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out_dir = out_dir or os.path.join(ROOT, "_build", "host_sanitized")
    os.makedirs(out_dir, exist_ok=True)
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + SANITIZE_FLAGS
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]

    def compile_one(src):
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        r = subprocess.run([hipcc] + flags + inc + ["-c", "-o", obj, src], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed on %s: %s" % (src, r.stderr[-4000:]))
        return obj

    with ThreadPoolExecutor(max_workers=len(SRC)) as ex:
        objs = list(ex.map(compile_one, SRC))
    lib = os.path.join(out_dir, "libddx.so")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + SANITIZE_FLAGS + ["-o", lib] + objs,
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s" % r.stderr[-4000:])
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
