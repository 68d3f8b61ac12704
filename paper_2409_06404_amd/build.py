"""Build the HIP/C++ library libcrf.so in-tree with hipcc for gfx950."""
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libcrf.so")
SOURCES = ["api.cpp", "mech.cpp", "kernels.hip"]


def hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build_library(arch="gfx950", verbose=False):
    """Compile every source for `arch` and link libcrf.so (always rebuilds)."""
    out_tmp = LIB + ".tmp"
    cmd = [hipcc(), "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={arch}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-result",
           "-o", out_tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(out_tmp, LIB)
    return LIB


def build_host_only_library(out, sanitize=True, verbose=False):
    """The host code (api.cpp, mech.cpp) with launchers that report a missing device
    (host_only.cpp), built by the host compiler alone: mechanisms load with device -1 and every
    call is validated, nothing computes.  With sanitize, the address and undefined-behaviour
    sanitizers are compiled in (every error fatal); a process that loads the result must
    preload the sanitizer runtime (host_sanitizer_runtime())."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    flags = ["-std=c++17", "-fPIC", "-g", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-result"]
    if sanitize:
        flags += ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    objs, procs = [], []
    for src in ("api.cpp", "mech.cpp", "host_only.cpp"):          # compiled side by side
        objs.append(out + "." + src + ".o")
        cmd = ["g++", "-c"] + flags + ["-o", objs[-1], os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd))
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    logs = [(p.communicate()[0], p.returncode) for p in procs]
    if any(rc != 0 for _, rc in logs):
        raise RuntimeError("g++ failed:\n" + "".join(t for t, rc in logs if rc != 0))
    cmd = ["g++", "-shared"] + flags + ["-o", out] + objs + ["-L", os.path.join(rocm, "lib"), "-lamdhip64",
                                                            "-Wl,-rpath," + os.path.join(rocm, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    for o in objs:
        os.remove(o)
    if r.returncode != 0:
        raise RuntimeError("g++ failed:\n" + r.stdout + r.stderr)
    return out


def host_sanitizer_runtime():
    """Path of the host compiler's address-sanitizer runtime (to preload), or None."""
    r = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


if __name__ == "__main__":
    print(build_library(verbose=True))
