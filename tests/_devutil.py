"""Helpers for the GPU tests: move a numpy CSR to device tensors and run the
library's walk entry points through the C ABI."""
import numpy as np
import torch

import paper_2110_06196_amd as n2v


def upload(O, D, W):
    Ot = torch.from_numpy(np.ascontiguousarray(O, dtype=np.uint64).view(np.int64)).cuda()
    Dt = torch.from_numpy(np.ascontiguousarray(D, dtype=np.int32)).cuda()
    Wt = None if W is None else torch.from_numpy(np.ascontiguousarray(W, dtype=np.uint32).view(np.int32)).cuda()
    g = n2v.n2v_graph_upload(Ot, Dt, Wt)
    return g, (Ot, Dt, Wt)


def run(g, starts, reps, L, kind, p=1.0, q=1.0, seed=0, base=0):
    S = torch.from_numpy(np.ascontiguousarray(starts, dtype=np.int32)).cuda()
    if kind == n2v.N2V_FIRST_ORDER:
        Y, lens = n2v.n2v_walks_first_order(g, S, reps, L, seed, base)
    else:
        Y, lens = n2v.n2v_walks_node2vec(g, S, reps, L, p, q, seed, base)
    torch.cuda.synchronize()
    return Y.cpu().numpy(), lens.cpu().numpy()
