"""Helpers for tests that load the built library."""
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ensure_built():
    from paper_2009_04604_amd import binding, build
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return binding


def declared_symbols():
    import re
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(lbm_\w+)\s*\(", txt, re.M)))
