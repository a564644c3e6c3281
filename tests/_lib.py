"""Test helpers: make sure the HIP library is built, compare fields."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ensure_built():
    from paper_1908_09235_amd import build
    if not build.up_to_date():
        build.build()


def header_symbols():
    with open(os.path.join(ROOT, "include", "lbm2p.h")) as f:
        txt = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(lbm_\w+)\s*\(", txt, re.M)))


def rel_err(a, b, mask):
    """max |a - b| / max |b| over the mask (the parity norm for rho and u)."""
    den = np.max(np.abs(b[mask]))
    if den == 0:
        return float(np.max(np.abs(a[mask])))
    return float(np.max(np.abs(a[mask] - b[mask])) / den)
