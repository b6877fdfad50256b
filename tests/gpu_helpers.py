"""Shared helpers of the GPU parity tests: run the HIP library and the oracle on the same
seeded inputs and compare what is unique (products X1 X2^T, residual histories)."""
import numpy as np

from oracle.lowrank import rel_distance
from oracle.spksm import spksm as oracle_spksm


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def gpu_ops(cfg):
    import paper_2311_16019_amd as skr
    A = skr.Operator.from_csr(cfg["A"].indptr, cfg["A"].indices, cfg["A"].data, diag=cfg.get("sigma"))
    B = skr.Operator.from_csr(cfg["B"].indptr, cfg["B"].indices, cfg["B"].data)
    return A, B


def to_dev(x):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def gpu_solve(cfg, **params):
    import paper_2311_16019_amd as skr
    A, B = gpu_ops(cfg)
    res = skr.solve(A, B, to_dev(cfg["C1"]), to_dev(cfg["C2"]), **params)
    torch_cuda().cuda.synchronize()
    return res, (A, B)


def oracle_solve(cfg, **params):
    params = dict(params)
    params.pop("precision", None)
    return oracle_spksm(cfg["A"], cfg["B"], cfg["C1"], cfg["C2"], sigma=cfg.get("sigma"), **params)


def product_distance(gpu_res, orc_res):
    X1 = gpu_res.X1.cpu().numpy()
    X2 = gpu_res.X2.cpu().numpy()
    return rel_distance(X1, X2, orc_res.X1, orc_res.X2)


def history_ratio(gpu_res, orc_res):
    gd = dict(gpu_res.history)
    od = dict(orc_res.history)
    common = sorted(set(gd) & set(od))
    return max(abs(gd[d] / od[d] - 1.0) for d in common) if common else float("nan")
