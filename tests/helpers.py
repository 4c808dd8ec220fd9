"""Shared test helpers: run the HIP path through the binding and compare with the oracle."""
import itertools
import re
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polydet.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(polydet_[a-z_]+)\s*\(", text)))


def box_to_dict(box):
    box = np.asarray(box, dtype=object)
    if box.ndim == 0:
        v = int(box[()])
        return {(): v} if v else {}
    return {tuple(int(x) for x in idx): int(box[idx]) for idx in np.ndindex(box.shape)
            if box[idx] != 0}


def supported_lanes(n):
    """(order, lanes) pairs with a compiled elimination kernel."""
    out = []
    if n <= 12:
        out.append(1)
    if 2 <= n <= 16:
        out.append(2)
    if 4 <= n <= 24:
        out.append(4)
    if 8 <= n <= 32:
        out.append(8)
    if 16 <= n <= 32:
        out.append(16)
    return out


def mont_to_plain(x, p):
    """x * 2^-32 mod p."""
    return int(x) * pow(1 << 32, p - 2, p) % p


def node_index(j, N):
    idx = 0
    for jj, nn in zip(j, N):
        idx = idx * nn + jj
    return idx
