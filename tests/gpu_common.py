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
    """sqrt(sum|a-b|^2 / sum|b|^2) over one or two component pairs (a printed
    figure; parity is asserted element by element with assert_elementwise)."""
    num = np.sum((a - b) ** 2)
    den = np.sum(b ** 2)
    if a2 is not None:
        num += np.sum((a2 - b2) ** 2)
        den += np.sum(b2 ** 2)
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def omega(mat, **kw):
    return O.omega_vector(mat.lame_lambda, mat.lame_mu, **kw)


def assert_elementwise(got, want, rtol: float, what: str = "", atol_frac: float = 0.1) -> float:
    """Element-wise parity of one field or a tuple of fields (e.g. (ux, uy)),
    each against its reference:
      max |got - want| <= rtol * max |want|                    (every element), and
      |got - want| <= rtol * |want| + atol_frac * rtol * max |want|  (per element),
    so a single element off by more than the bar fails even in a large field.
    Returns the worst max-norm ratio and prints it with the L2 ratio."""
    gots = got if isinstance(got, (tuple, list)) else (got,)
    wants = want if isinstance(want, (tuple, list)) else (want,)
    scale = max(float(np.max(np.abs(np.asarray(w)))) for w in wants)
    if scale == 0.0:
        scale = 1.0
    worst, num, den = 0.0, 0.0, 0.0
    for k, (g, w) in enumerate(zip(gots, wants)):
        g = np.asarray(g, np.float64)
        w = np.asarray(w, np.float64)
        assert g.shape == w.shape, (what, g.shape, w.shape)
        err = np.abs(g - w)
        assert np.all(np.isfinite(g)), f"{what}[{k}]: non-finite values"
        worst = max(worst, float(err.max()) / scale)
        bad = err > rtol * np.abs(w) + atol_frac * rtol * scale
        if bad.any():
            i = np.unravel_index(int(np.argmax(np.where(bad, err, -1.0))), err.shape)
            raise AssertionError(
                f"{what}[{k}]: {int(bad.sum())} of {bad.size} elements beyond "
                f"{rtol:g}*|ref| + {atol_frac * rtol:g}*max|ref|; worst at {i}: got {g[i]!r}, "
                f"want {w[i]!r}")
        num += float(np.sum(err ** 2))
        den += float(np.sum(w ** 2))
    assert worst <= rtol, f"{what}: max|d|/max|ref| = {worst:.3e} > {rtol:g}"
    say(f"  parity {what}: max|d|/max|ref| {worst:.2e}, rel L2 "
        f"{np.sqrt(num / den) if den > 0 else 0.0:.2e} (bar {rtol:g})")
    return worst
