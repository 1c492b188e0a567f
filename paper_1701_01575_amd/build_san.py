"""A host-sanitized build of libdsa.so for CPU test runs: AddressSanitizer
and UndefinedBehaviorSanitizer on the host code only (argument checks,
planning, ingest); the device code is built as usual.  The result is loaded
through DSA_LIBRARY by a process that preloads clang's sanitizer runtime."""
from __future__ import annotations

import os

from . import build as B

HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-shared-libasan"]


def build(out_dir: str) -> str:
    return B.build(extra_flags=HOST_SANITIZE, lib_path=os.path.join(out_dir, "libdsa_san.so"))
