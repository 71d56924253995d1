"""Locate (building if absent) the HIP library for the tests."""
import os

from paper_2506_11586_amd import build as _build


def ensure_built() -> str:
    if not os.path.exists(_build.LIB):
        _build.build()
    return _build.LIB
