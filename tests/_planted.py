"""Planted mistakes: copies of the oracle source with one deliberate slip, compiled on the CPU, so
that a pin can show it fails for that slip (a pin that passes for a plausible mistake pins nothing).
"""
import os

from oracle import oracle as orc


def oracle_source():
    with open(orc.SRC) as fh:
        return fh.read()


def variant(tmp_dir, tag, replacements):
    """Build the oracle with each (old, new) text replacement applied exactly once; returns a
    context manager under which the `oracle.oracle` functions call that variant."""
    src = oracle_source()
    for old, new in replacements:
        n = src.count(old)
        assert n == 1, f"planted mistake '{tag}': pattern found {n} times"
        src = src.replace(old, new)
    path = orc.build_variant(src, str(tmp_dir), tag)
    assert os.path.exists(path)
    return orc.using_library(path)
