"""The entry point that allocates nothing (pbmp_site_fields_noalloc)
against pbmp_site_fields on the same context, through the C-ABI: two calls
in a row, the second on a smaller mesh and site set, each equal to the
existing entry point's output (the same kernels; the partial sums may be
split into fewer chunks, so the bar is relative 1e-12 in FP64 and 1e-6 in
mixed precision, far below the oracle bars of the site readout).  Named to
be collected last."""

import numpy as np
import pytest

from synth import workload

pytestmark = pytest.mark.gpu


def _solver(w, precision, mode):
    from paper_1810_03698_amd import Solver
    s = Solver(eps_in=1.0, eps_out=80.0, kappa=0.125, precision=precision, mode=mode)
    s.set_mesh(w["verts"], w["tris"])
    s.set_sites(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"])
    return s


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_noalloc_site_fields_match_allocating_entry_point(precision, tol):
    import torch
    dev = torch.device("cuda:0")
    for k, (name, mode) in enumerate((("globule_1000", "treecode"), ("sphere_1280", "direct"))):
        w = workload(name)
        s = _solver(w, precision, mode)
        n = len(w["tris"])
        x = np.random.default_rng(60 + k).normal(size=2 * n)
        ref = s.site_fields(x)
        xd = torch.as_tensor(x, dtype=torch.float64, device=dev)
        out = torch.full((len(w["q"]), 10), float("nan"), dtype=torch.float64, device=dev)
        s.site_fields_noalloc(xd, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(name, precision, "sites", len(w["q"]), "panels", n, "max rel err", err)
        assert np.isfinite(got).all()
        assert err < tol
        s.close()


def test_noalloc_rejects_host_pointers():
    from paper_1810_03698_amd import Solver
    w = workload("sphere_1280")
    s = _solver(w, "fp64", "direct")
    with pytest.raises(ValueError):
        s.site_fields_noalloc(np.zeros(2 * len(w["tris"])), np.zeros((len(w["q"]), 10)))
    s.close()
