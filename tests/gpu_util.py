"""Shared helpers of the GPU tests (not collected by pytest)."""
import sys

import numpy as np

TREE_KEYS = ["perm", "level", "morton", "first", "count", "parent", "child_begin", "nchild",
             "U_off", "U_src", "V_off", "V_src", "W_off", "W_src", "X_off", "X_src"]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def to_dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def gpu_solve(x, q, p, **kw):
    from paper_2508_02626_amd import fmm
    pl = fmm.Plan(to_dev(x), p, **kw)
    phi, fld = pl.evaluate(to_dev(q))
    return pl, phi.cpu().numpy(), fld.cpu().numpy()


def oracle_tree(x, **kw):
    import oracle
    # (options of the GPU path only, such as the M2L method, do not change the tree)
    return oracle.Tree(x, root=kw.get("root"), uniform_depth=kw.get("uniform_depth", -1),
                       max_depth=kw.get("max_depth", 21), leaf_size=kw.get("leaf_size", 64))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
