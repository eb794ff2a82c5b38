"""The paper's accuracy experiment (Sec. V-A) at a small size, on the GPU path:
known spectra, FP64 dense -> band on the host, band -> bidiagonal on the GPU in
FP64 / FP32 / FP16, sigma by the device bisection, relative error
||sigma_hat - sigma|| / ||sigma|| against the prescribed sigma."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2510_12705_amd import accuracy as acc  # noqa: E402


@pytest.mark.parametrize("kind", acc.SPECTRA)
def test_known_spectrum_errors(kind):
    from paper_2510_12705_amd import bb
    bb.reset_params()
    n, b = 768, 48
    out = {}
    for trial in range(2):
        band, s = acc.test_matrix(kind, n, b, seed=trial)
        for p in ("fp64", "fp32", "fp16"):
            rel, mx = acc.errors(acc.gpu_sigma(band, n, b, p), s)
            out.setdefault(p, []).append(rel)
    print("%s n=%d b=%d: %s" % (kind, n, b, ", ".join("%s %.2e" % (p, max(v)) for p, v in out.items())), flush=True)
    sys.stdout.flush()
    assert max(out["fp64"]) <= 20 * n * np.finfo(np.float64).eps
    assert max(out["fp32"]) <= 50 * n * np.finfo(np.float32).eps
    assert max(out["fp16"]) <= 5e-2
