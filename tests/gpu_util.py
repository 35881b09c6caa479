"""Helpers shared by the GPU tests: run the HIP sort and compare with the oracle."""
import numpy as np
import torch

import oracle
from paper_1305_1157_amd import gen, s5

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gpu_sort(chars, offs, cfg=None):
    # keep at least one aligned word of arena so a zero-length arena still has storage
    c = chars if chars.size else np.zeros(8, np.uint8)
    perm, lcp = s5.sort(to_dev(c), to_dev(offs.astype(np.uint64)), cfg=cfg)
    torch.cuda.synchronize()
    return perm.cpu().numpy(), lcp.cpu().numpy()


def assert_parity(chars, offs, cfg=None, label=""):
    perm, lcp = gpu_sort(chars, offs, cfg)
    ref_perm, ref_lcp = oracle.sort(chars, offs)
    if not np.array_equal(perm, ref_perm):
        bad = np.nonzero(perm != ref_perm)[0]
        raise AssertionError(f"{label}: perm differs at {bad.size} positions, first {bad[:8]}")
    if not np.array_equal(lcp, ref_lcp):
        bad = np.nonzero(lcp != ref_lcp)[0]
        raise AssertionError(f"{label}: lcp differs at {bad.size} positions, first {bad[:8]} "
                             f"got {lcp[bad[:8]]} want {ref_lcp[bad[:8]]}")
    return s5.stats()


def strings_parity(strings, cfg=None, label=""):
    chars, offs = gen.from_strings(strings)
    return assert_parity(chars, offs, cfg, label)
