"""Build libccm and tests/native/host_stress.cpp with the host code
instrumented by a sanitizer (the device code is not: GPU sanitizers are
not used here).

    python tests/native/build_sanitized.py address OUTDIR
    python tests/native/build_sanitized.py thread OUTDIR

writes OUTDIR/libccm_<kind>.so and OUTDIR/host_stress_<kind>; run the
latter from the repository root on a machine with the GPU, e.g.
ASAN_OPTIONS=detect_leaks=0 OUTDIR/host_stress_address.  In the library's
hipcc lines every -fsanitize flag goes to the host compilation only
(-Xarch_host); the driver has no device code and is built by clang++.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_1905_00565_amd import build as B  # noqa: E402


def main():
    kind, out = sys.argv[1], os.path.abspath(sys.argv[2])
    if kind not in ("address", "thread"):
        raise SystemExit("kind must be address or thread")
    os.makedirs(out, exist_ok=True)
    san = ["-Xarch_host", f"-fsanitize={kind}", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xarch_host", "-g"]
    jobs = [(src, os.path.join(out, os.path.basename(obj)), list(extra) + san)
            for src, obj, extra in B.units()]
    with ThreadPoolExecutor(max_workers=B.jobs()) as ex:
        objs = list(ex.map(lambda j: B.compile_unit(*j), jobs))
    lib = os.path.join(out, f"libccm_{kind}.so")
    link = [B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *san, "-o", lib, *objs]
    subprocess.run(link, check=True)
    # the driver is plain C++ (no device code): ROCm's clang++ directly
    exe = os.path.join(out, f"host_stress_{kind}")
    clang = os.path.join(os.path.dirname(os.path.realpath(B.hipcc())), "..", "llvm", "bin",
                         "clang++")
    drv = [os.path.normpath(clang), "-O1", "-std=c++17", f"-fsanitize={kind}",
           "-fno-omit-frame-pointer", "-g", f"-I{B.INCLUDE}",
           os.path.join(HERE, "host_stress.cpp"), "-o", exe, lib, f"-Wl,-rpath,{out}",
           "-lpthread"]
    subprocess.run(drv, check=True)
    for o in objs:
        os.remove(o)
    print(exe)


if __name__ == "__main__":
    main()
