"""Helpers shared by the GPU tests: moving numpy arrays to the device and back."""
import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(a: np.ndarray):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t) -> np.ndarray:
    return t.cpu().numpy()


def padded_rows(a: np.ndarray, ld: int, offset: int = 0, fill: int = 0xA5):
    """Device tensor whose rows are `ld` bytes apart, data starting `offset` bytes into the buffer.

    Returns (base tensor, 2-D row view)."""
    torch = torch_cuda()
    rows, L = a.shape
    base = torch.full((offset + max(rows, 1) * ld + 16,), fill, dtype=torch.uint8, device="cuda")
    view = base[offset:offset + rows * ld].view(rows, ld)[:, :L] if rows else base[:0].view(0, L)
    if rows:
        view.copy_(torch.from_numpy(np.ascontiguousarray(a)).to("cuda"))
    return base, view
