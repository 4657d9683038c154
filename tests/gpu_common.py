"""Helpers shared by the GPU tests (host-side marshalling only)."""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(a, b, a2=None, b2=None) -> float:
    """sqrt(sum|a-b|^2 / sum|b|^2) over one or two component pairs."""
    num = np.sum((a - b) ** 2)
    den = np.sum(b ** 2)
    if a2 is not None:
        num += np.sum((a2 - b2) ** 2)
        den += np.sum(b2 ** 2)
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def omega(mat, **kw):
    return O.omega_vector(mat.lame_lambda, mat.lame_mu, **kw)
