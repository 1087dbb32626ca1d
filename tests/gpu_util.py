"""Host/device marshalling helpers for the GPU tests (no arithmetic of the method)."""
import numpy as np
import torch


def dev(a: np.ndarray) -> torch.Tensor:
    """Copy a uint32/uint64 numpy array to the GPU (stored as int32/int64 bits)."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32).copy()).cuda()
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64).copy()).cuda()
    raise TypeError(a.dtype)


def host(t: torch.Tensor, dtype) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().view(dtype)


def rev(j: int, l: int) -> int:
    return int(format(j, f"0{l}b")[::-1], 2) if l else 0
