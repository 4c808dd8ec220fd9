"""Shared test helpers: run the HIP path through the binding and compare with the oracle."""
import itertools
import re
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    """Every polydet_* function declared in the headers under include/."""
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if h.endswith(".h"):
            text = open(os.path.join(INCLUDE, h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names.update(re.findall(r"\b(polydet_[a-z_]+)\s*\(", text))
    return sorted(names)


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


Q31 = 2147483629  # a prime below 2^31 that is not of the NTT form used by the library


def limbs_mod_q(limbs, q):
    """Two's-complement little-endian uint32 limb rows -> values mod q (vectorised)."""
    limbs = np.asarray(limbs).view(np.uint32).astype(np.uint64)
    L = limbs.shape[1]
    acc = np.zeros(limbs.shape[0], dtype=np.uint64)
    for l in range(L):
        acc = (acc + (limbs[:, l] % q) * np.uint64(pow(2, 32 * l, q))) % q
    neg = (limbs[:, L - 1] >> np.uint64(31)).astype(bool)
    wrap = np.uint64(pow(2, 32 * L, q))
    acc[neg] = (acc[neg] + np.uint64(q) - wrap) % q
    return acc


def eval_box_mod_q(vals, box, point, q):
    """sum_e vals[e] prod_v point_v^{e_v} mod q for a dense box (first variable slowest)."""
    arr = vals.reshape(box) if box else vals.reshape(())
    for v in range(len(box) - 1, -1, -1):
        pw = np.array([pow(int(point[v]), e, q) for e in range(box[v])], dtype=np.uint64)
        arr = (arr * pw) % q
        arr = np.sum(arr, axis=-1, dtype=np.uint64) % q if arr.ndim else arr
    return int(arr)


def device_values_at_point(d_out, off, C, L, box, point, q):
    """The output polynomial (limbs on the device) reduced mod q and evaluated at `point`,
    with torch int64 arithmetic on the device (every product stays below 2^62)."""
    import torch
    limbs = d_out[off:off + C * L].view(C, L).to(torch.int64) & 0xFFFFFFFF
    acc = torch.zeros(C, dtype=torch.int64, device=d_out.device)
    for l in range(L):
        acc = (acc + (limbs[:, l] % q) * pow(2, 32 * l, q)) % q
    neg = (limbs[:, L - 1] >> 31) == 1
    acc = torch.where(neg, (acc + q - pow(2, 32 * L, q)) % q, acc)
    arr = acc.view(box) if box else acc.view(())
    for v in range(len(box) - 1, -1, -1):
        pw = torch.tensor([pow(int(point[v]), e, q) for e in range(box[v])], dtype=torch.int64,
                          device=d_out.device)
        arr = (arr * pw) % q
        arr = arr.sum(dim=-1) % q if arr.dim() else arr  # at most 161 terms < 2^31 each
    return int(arr.item())


def det_mod_q_stack(A, q):
    """Determinants mod q of a stack of matrices (numpy uint64 [count, n, n], entries < q) by
    Gaussian elimination with the first nonzero pivot, vectorised over the stack."""
    A = A.copy()
    count, n, _ = A.shape
    det = np.ones(count, dtype=np.uint64)
    alive = np.ones(count, dtype=bool)
    idx = np.arange(count)
    for k in range(n):
        nz = A[:, k:, k] != 0
        has = nz.any(axis=1)
        alive &= has
        r = k + np.argmax(nz, axis=1)
        swap = (r != k) & has
        rows_k = A[idx, k].copy()
        A[idx, k] = A[idx, r]
        A[idx, r] = rows_k
        det = np.where(swap, (q - det) % q, det)
        piv = np.where(has, A[:, k, k], 1).astype(np.uint64)
        det = det * piv % q
        inv = np.ones(count, dtype=np.uint64)
        base, e = piv.copy(), q - 2
        while e:
            if e & 1:
                inv = inv * base % q
            base = base * base % q
            e >>= 1
        for i in range(k + 1, n):
            f = A[:, i, k] * inv % q
            A[:, i, k:] = (A[:, i, k:] + (q - f)[:, None] * A[:, k, k:]) % q
    return np.where(alive, det, 0)
