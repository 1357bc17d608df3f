"""SHA-256 of the sources liblks.so is built from.

build() compiles it into the library (lks_source_digest), and the binding
refuses a library whose digest differs from the sources next to it, so a
stale build is never tested or timed by mistake.
"""
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "lks_kernels.hip"),
           os.path.join(HERE, "csrc", "lks_api.hip"),
           os.path.join(HERE, "csrc", "lks_internal.h"),
           os.path.join(ROOT, "include", "lks.h")]


def source_digest():
    """Hex digest over the library's sources, or None if any is missing."""
    h = hashlib.sha256()
    for path in SOURCES:
        if not os.path.exists(path):
            return None
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode())
            h.update(f.read())
    return h.hexdigest()
