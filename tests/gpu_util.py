"""Helpers shared by the GPU parity tests (no solver arithmetic here)."""
import numpy as np
import torch


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    """max |got - ref| / max |ref| over all nodes."""
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def banner(msg: str):
    print("[gpu-case] " + msg, flush=True)
