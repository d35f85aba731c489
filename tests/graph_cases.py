"""Shared sequence of the graph replay test (parent and child process)."""
import numpy as np

import h2inputs


def run_sequence(P):
    import torch
    x = h2inputs.points("cube", 1536, 11)
    sc = h2inputs.kernel_scale("1/(4piN)", 1536)
    h = P.h2_build(x, sc, 1.0, 32, 3, 1e-8, 27)
    f = P.h2_factor_S(P.h2_sparsify(h, P.H2_MIXED))
    outs = []
    rng = np.random.default_rng(21)
    for rep in range(3):
        b = rng.standard_normal((1536, 3))
        bd = torch.from_numpy(np.ascontiguousarray(b.T)).cuda().T
        xd = torch.zeros_like(bd)
        P.h2_apply_inverse(f, bd, xd)
        torch.cuda.synchronize()
        outs.append(xd.cpu().numpy())
        yd = torch.zeros_like(bd)
        P.h2_matvec(h, bd, yd)
        torch.cuda.synchronize()
        outs.append(yd.cpu().numpy())
        # eager work of the program between the replays
        (bd * 2.0).sum().item()
    return np.stack(outs)
