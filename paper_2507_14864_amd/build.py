"""Build ``libfj.so`` (HIP, gfx950) from ``csrc/*.hip``.

Every HIP source is compiled with packed-FP32 instruction generation turned
off (``-Xclang -target-feature -Xclang -packed-fp32-ops``).
"""
import glob
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
ARCH = "gfx950"


def hip_flags():
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, jobs: int = 8) -> str:
    srcs = sorted(glob.glob(os.path.join(_HERE, "csrc", "*.hip")))
    objdir = os.path.join(_HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in srcs:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = ["hipcc", *hip_flags(), "-c", src, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    errors = []
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            errors.append(" ".join(cmd) + "\n" + text)
        elif verbose and text.strip():
            print(text)
    if errors:
        raise RuntimeError("HIP build failed:\n" + "\n".join(errors))
    out = os.path.join(_HERE, "libfj.so")
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out + ".tmp"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
