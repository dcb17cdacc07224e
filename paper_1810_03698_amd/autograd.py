"""torch.autograd.Function around the library: forward = pbmp_solve,
backward = pbmp_backward (the adjoint kernels).  PyTorch only carries the
tensors; all arithmetic runs in libpbmp.so."""

import torch

from .pbmp import Solver


class SolvationEnergy(torch.autograd.Function):
    """dG(verts, xyz, q, d, Q9) in kcal/mol for a fixed triangle topology and
    fixed polarisabilities."""

    @staticmethod
    def forward(ctx, solver, verts, tris, xyz, q, d, Q9, alpha):
        solver.set_mesh(verts.detach().contiguous(), tris.contiguous())
        solver.set_sites(xyz.detach().contiguous(), q.detach().contiguous(),
                         d.detach().contiguous(), Q9.detach().contiguous(),
                         alpha.detach().contiguous())
        r = solver.solve(outputs=False)
        ctx.solver = solver
        ctx.state_id = solver.state_id
        ctx.device = xyz.device
        return torch.tensor(r["dG"], dtype=torch.float64, device=xyz.device)

    @staticmethod
    def backward(ctx, grad_out):
        if ctx.solver.state_id != ctx.state_id:
            # the library differentiates the solver's current state: a later
            # set_mesh / set_sites / solve on the same solver replaced the
            # state this energy came from
            raise RuntimeError(
                "solvation_energy: the Solver was used again after this energy was "
                "computed (its mesh, sites or solution changed); use one Solver per "
                "energy that is differentiated")
        need_v = ctx.needs_input_grad[1]
        dev = ctx.device if ctx.device.type == "cuda" else None
        g = ctx.solver.backward(float(grad_out), verts=need_v, device=dev)
        conv = lambda a: a if isinstance(a, torch.Tensor) else torch.as_tensor(a)
        gv = conv(g["verts"]) if need_v else None
        return (None, gv, None, conv(g["xyz"]), conv(g["q"]), conv(g["d"]),
                conv(g["Q9"]).reshape(-1, 9), None)


def solvation_energy(verts, tris, xyz, q, d, Q9, alpha, solver=None, **options):
    """Differentiable solvation energy (kcal/mol).  `options` are Solver
    keyword arguments (precision, mode, tolerances, ...)."""
    solver = solver or Solver(**options)
    return SolvationEnergy.apply(solver, verts, tris, xyz, q, d, Q9.reshape(-1, 9), alpha)
