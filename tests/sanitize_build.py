"""Host-sanitized builds for the CPU suite: the library with AddressSanitizer
and UndefinedBehaviorSanitizer on its host code (device code is compiled as
usual), and the oracle with the same sanitizers, both against clang's shared
sanitizer runtime so that one runtime serves the whole test process.  Used by
tests/test_sanitize.py only; no GPU run loads these builds."""
from __future__ import annotations

import glob
import os

HOST_SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer", "-shared-libsan"]
CLANG = "/opt/rocm/llvm/bin/clang"


def runtime() -> str:
    """clang's shared AddressSanitizer runtime (preloaded into the test process)."""
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found under /opt/rocm/llvm")
    return found[-1]


def build_library(outdir: str) -> str:
    import importlib
    B = importlib.import_module("paper_2412_08308_amd.build")
    flags = []
    for f in HOST_SAN:
        flags += ["-Xarch_host", f]
    return B.build(out=os.path.join(outdir, "libswdb.so"), extra=flags + ["-Xarch_host", "-g"], link_extra=flags)


def build_oracle(outdir: str) -> str:
    import importlib
    O = importlib.import_module("oracle.build")      # the module (the package re-exports its function)
    return O.build(out=os.path.join(outdir, "liboracle.so"), cc=CLANG, extra=HOST_SAN + ["-g"])
