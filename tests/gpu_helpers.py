"""Shared helpers of the GPU tests (device transfer and error metrics)."""
import numpy as np
import pytest
import torch


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2209_15040_amd import binding
    return binding


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).cuda()


def to_host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(a, b) -> float:
    """||a - b|| / ||b|| over all re and im components, in FP64."""
    a = np.asarray(a).ravel().astype(np.complex128)
    b = np.asarray(b).ravel().astype(np.complex128)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def c16_to_c128(t: torch.Tensor, kind: str) -> np.ndarray:
    """(..., 2) float16 / bfloat16 device tensor to complex128 (exact)."""
    torch.cuda.synchronize()
    if kind == "fp16":
        p = t.cpu().numpy().astype(np.float64)
    else:
        p = t.cpu().view(torch.int16).numpy().view(np.uint16)
        p = (p.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return p[..., 0] + 1j * p[..., 1]


def c16_to_dev(pairs: np.ndarray, kind: str) -> torch.Tensor:
    if kind == "fp16":
        return torch.from_numpy(np.ascontiguousarray(pairs)).cuda()
    return torch.from_numpy(np.ascontiguousarray(pairs).view(np.int16)).view(torch.bfloat16).cuda()
