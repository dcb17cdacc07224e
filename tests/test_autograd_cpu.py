"""The autograd wrapper refuses to differentiate a solver whose state was
replaced after the forward pass (a second energy computed on the same
Solver before .backward()).  CPU only: a stand-in object with the Solver's
call surface replaces the library."""

import numpy as np
import pytest
import torch

from paper_1810_03698_amd.autograd import SolvationEnergy


class _FakeSolver:
    def __init__(self):
        self.state_id = 0
        self.backward_calls = 0

    def set_mesh(self, verts, tris):
        self.state_id += 1

    def set_sites(self, xyz, q, d, Q9, alpha):
        self.state_id += 1
        self.q = np.asarray(q)

    def solve(self, outputs=True):
        self.state_id += 1
        return {"dG": float(np.sum(self.q ** 2))}

    def backward(self, dG_bar=1.0, verts=True, device=None):
        self.backward_calls += 1
        m = len(self.q)
        return {"xyz": np.zeros((m, 3)), "q": 2 * dG_bar * self.q, "d": np.zeros((m, 3)),
                "Q9": np.zeros((m, 9)), "verts": np.zeros((4, 3))}


def _inputs(scale):
    t = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)
    verts = t(np.zeros((4, 3)))
    tris = torch.zeros((4, 3), dtype=torch.int32)
    return verts, tris, t(np.zeros((2, 3))), t(scale * np.array([1.0, -2.0])), \
        t(np.zeros((2, 3))), t(np.zeros((2, 9))), torch.ones(2, dtype=torch.float64)


def test_backward_of_the_current_state_works():
    s = _FakeSolver()
    v, tr, xyz, q, d, Q9, a = _inputs(1.0)
    e = SolvationEnergy.apply(s, v, tr, xyz, q, d, Q9, a)
    e.backward()
    assert np.allclose(q.grad.numpy(), [2.0, -4.0])


def test_backward_after_reuse_raises():
    s = _FakeSolver()
    v, tr, xyz, q, d, Q9, a = _inputs(1.0)
    e1 = SolvationEnergy.apply(s, v, tr, xyz, q, d, Q9, a)
    v2, tr2, xyz2, q2, d2, Q92, a2 = _inputs(3.0)
    e2 = SolvationEnergy.apply(s, v2, tr2, xyz2, q2, d2, Q92, a2)
    with pytest.raises(RuntimeError, match="used again"):
        e1.backward()
    assert s.backward_calls == 0
    e2.backward()  # the solver's current state is e2's
    assert np.allclose(q2.grad.numpy(), [6.0, -12.0])
