"""md_kinetic_energy_noalloc (no context, partial sums in the library's own per-GPU array) against
md_kinetic_energy (partial sums in the context's scratch): two calls in a row, the second with a smaller input,
each equal to the context path bit for bit and to numpy's float64 sum to 1e-12."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_kinetic_energy_noalloc_matches_context_path():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1912_04232_amd import md
    md.load()
    ctx = md.Context()
    rng = np.random.default_rng(2027)
    for n, dim in ((300001, 3), (4099, 2)):
        print(f"noalloc kinetic energy: N={n} dim={dim}", file=sys.stderr, flush=True)
        v = rng.standard_normal((n, dim)).astype(np.float32)
        vd = torch.as_tensor(v, device=ctx.device)
        want = torch.full((1,), -1.0, dtype=torch.float64, device=ctx.device)
        got = torch.full((1,), -2.0, dtype=torch.float64, device=ctx.device)
        md.kinetic_energy(ctx, vd, want)
        md.kinetic_energy_noalloc(vd, got)
        torch.cuda.synchronize()
        ref = 0.5 * math.fsum((v.astype(np.float64) ** 2).ravel().tolist())
        assert float(got.item()) == float(want.item())
        assert float(got.item()) == pytest.approx(ref, rel=1e-12)
