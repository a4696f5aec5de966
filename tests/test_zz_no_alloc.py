"""pdf_cfl_dt_noalloc (the entry point that allocates nothing) against pdf_cfl_dt through
the C ABI: bit-identical time steps on two calls in a row, the second on a smaller
problem, with the output in caller-owned device memory."""
import sys

import numpy as np
import pytest

from paper_1006_0532_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_cfl_noalloc_matches_the_allocating_call():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    from paper_1006_0532_amd import pdfgpu
    pdfgpu.load()
    _say("test_cfl_noalloc_matches_the_allocating_call")
    # a batched ensemble: problem 0 with 40x50 quads, problem 1 with 6x8 quads
    big = W.channel_small()
    small = W.channel_small(nx=6, ny=8)
    grids = [pdfgpu.Grid(m, f, mo) for (m, f, mo, _) in (big, small)]
    ini = [dict(big[3], ppe=20), dict(small[3], ppe=30, seed=big[3]["seed"])]
    e = pdfgpu.Ensemble(grids, ini)
    e.step([1e-3, 1e-3], 2)
    out = torch.full((4,), -1.0, dtype=torch.float64, device="cuda")
    for k, (problem, cfl) in enumerate([(0, 0.7), (1, 0.5)]):
        _say(f"  call {k}: problem {problem}, {(big, small)[problem][0].n_nodes} nodes")
        e.cfl_dt_noalloc(out.data_ptr() + 8 * k, cfl=cfl, problem=problem)
        torch.cuda.synchronize()
        ref = e.cfl_dt(cfl=cfl, problem=problem)
        got = float(out[k].item())
        assert ref > 0.0
        assert got == ref, (problem, got, ref)
    assert float(out[2].item()) == -1.0 and float(out[3].item()) == -1.0
    # bad arguments are refused before any device work
    with pytest.raises(pdfgpu.PdfError) as ex:
        e.cfl_dt_noalloc(out.data_ptr(), cfl=-1.0)
    assert ex.value.status == -1
    with pytest.raises(pdfgpu.PdfError) as ex:
        e.cfl_dt_noalloc(0, cfl=0.7)
    assert ex.value.status == -1
