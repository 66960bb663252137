"""Shared helpers of the GPU tests: build matching library and oracle MultiFabs
from the same box list and global input, and compare their valid cells."""
import numpy as np
import torch

from oracle import oracle as O


def lib():
    from paper_1604_03570_amd import boxtile as bt
    return bt


def say(msg: str) -> None:
    print(f"[gpu-test] {msg}", flush=True)


def make_pair(boxes, domain, periodic, ncomp, ng, dtype, g0, ghost_value=0.0):
    """Library MultiFab pair (ghosts set to ghost_value, valid = g0) and the oracle MultiFab."""
    bt = lib()
    ba = bt.BoxArray.from_boxes(boxes, domain, periodic)
    a = bt.MultiFab(ba, ncomp, ng, dtype)
    b = bt.MultiFab(ba, ncomp, ng, dtype)
    a.set_val(ghost_value, with_ghosts=True)
    b.set_val(ghost_value, with_ghosts=True)
    a.from_global(g0)
    o = O.OracleMultiFab(boxes, domain, periodic, ncomp, ng)
    o.data[...] = ghost_value
    o.load_global(np.asarray(g0, dtype=np.float64))
    torch.cuda.synchronize()
    return ba, a, b, o


def gpu_global(mf) -> np.ndarray:
    return mf.to_global().double().cpu().numpy()


def rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    m = np.isfinite(ref)
    return float(np.abs(got[m] - ref[m]).max() / np.abs(ref[m]).max())
