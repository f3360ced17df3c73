"""Build tests/c_abi_client (a C program on the library's C ABI and the FP64 oracle).

Run by __graft_entry__.build() after libsal.so and liboracle.so exist; the GPU test
tests/test_gpu_c_abi.py runs the binary.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "c_abi_client.c")
OUT = os.path.join(HERE, "c_abi_client")


def build(out: str = OUT) -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["gcc", "-O2", "-Wall", "-std=c11", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"),
           SRC, "-o", out + ".tmp",
           "-L", os.path.join(ROOT, "paper_1901_11095_amd"), "-l:libsal.so",
           "-L", os.path.join(ROOT, "oracle"), "-l:liboracle.so",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/../paper_1901_11095_amd:$ORIGIN/../oracle:" + os.path.join(rocm, "lib")]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())
