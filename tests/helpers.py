"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import numpy as np

from paper_2010_13213_amd import inputs


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_solve(ctx, problem, precision="fp64", report=False):
    """Solve through the C ABI; returns the host field (n_comp, n_cells)."""
    import torch
    from paper_2010_13213_amd import lgf
    plan = lgf.Plan.for_problem(ctx, problem, precision)
    f = torch.from_numpy(problem.flat_source()).cuda()
    out = plan.solve(f, report=report)
    torch.cuda.synchronize()
    u, rep = out if report else (out, None)
    res = u.cpu().numpy().reshape(problem.n_components, -1)
    plan.close()
    return (res, rep) if report else res


def level_cells(problem, k=0):
    return inputs.cell_coords(problem.levels[k].blocks, problem.nb)
