"""Hash of the library's sources (HIP files, their headers, the C header and
the compile flags): build.py compiles it into librwtrsv.so and _lib.load()
refuses a library whose hash differs from the sources next to it."""
from __future__ import annotations

import glob
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def source_files() -> list[str]:
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) +
                   glob.glob(os.path.join(HERE, "csrc", "*.hpp")))
    files.append(os.path.join(ROOT, "include", "rwtrsv.h"))
    return files


def source_hash(flags: list[str]) -> str | None:
    """16 hex digits, or None when the sources are not present."""
    files = source_files()
    if not all(os.path.exists(f) for f in files) or len(files) < 2:
        return None
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.relpath(f, ROOT).encode())
        h.update(b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]
