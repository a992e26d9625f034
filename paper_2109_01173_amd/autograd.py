"""torch.autograd wrappers of the MO-PCG solve and of IMEX Euler rollouts.

Every arithmetic step of the backward passes runs in the library:

* the multiterm operator is symmetric, so the adjoint of an elliptic solve
  is a second MO-PCG solve with the same operator and preconditioner
  (mofem_pcg_solve);
* the transpose of the full-node load M3[I, :] F M[:, I] (eq. (74)) is a
  full-output operator, dJ/dF = M3[:, I] Lambda M[I, :] (mofem_op_apply);
* dJ/dgamma = -<Lambda, M3 U M> and the batch sums of per-item gradients are
  Frobenius products (mofem_dot_accumulate);
* one reverse IMEX step is mofem_imex_adjoint_step.

Long rollouts keep the state every `checkpoint` steps; the backward pass
recomputes one segment at a time from its checkpoint (the forward solver is
deterministic, so the recomputed states equal the forward ones bit for bit)
and runs the reverse steps over it.  Memory: (steps / checkpoint +
checkpoint) states instead of one per step.
"""
import torch

from . import mofem as mf


class EllipticSolve(torch.autograd.Function):
    """U = L_gamma^{-1}(M3[I, :] F M[:, I]) for a batch of full-node loads F
    (batch, n, n); gamma is a 0-dim tensor equal to problem.gamma (the
    operator's bands are built with it)."""

    @staticmethod
    def forward(ctx, F, gamma, problem, tol=1e-10, maxit=500, flags=0):
        if float(gamma) != problem.gamma:
            raise ValueError("gamma differs from the operator's gamma (%r vs %r)" % (float(gamma), problem.gamma))
        F = F.contiguous()
        rhs = problem.rhs_op.apply(F)
        U = torch.empty_like(rhs)
        mf.pcg_solve(problem.op, problem.prec, rhs, U, tol=tol, maxit=maxit, flags=flags | mf.PCG_ZERO_GUESS)
        ctx.problem, ctx.tol, ctx.maxit, ctx.flags = problem, tol, maxit, flags
        ctx.save_for_backward(U)
        return U

    @staticmethod
    def backward(ctx, gU):
        (U,) = ctx.saved_tensors
        P = ctx.problem
        gU = gU.contiguous()
        Lam = torch.empty_like(gU)
        mf.pcg_solve(P.op, P.prec, gU, Lam, tol=ctx.tol, maxit=ctx.maxit, flags=ctx.flags | mf.PCG_ZERO_GUESS)
        dF = P.rhs_adjoint_op.apply(Lam) if ctx.needs_input_grad[0] else None
        dgamma = None
        if ctx.needs_input_grad[1]:
            MU = P.mass.apply(U)
            out = torch.zeros(1, dtype=torch.float64, device=U.device)
            # gamma is shared by the batch: one product over all items
            mf.dot_accumulate(Lam.reshape(1, -1), MU.reshape(1, -1), out, alpha=-1.0)
            dgamma = out.reshape(())
        return dF, dgamma, None, None, None, None


class ImexRollout(torch.autograd.Function):
    """`nsteps` IMEX Euler steps (mofem_imex_step) from state0
    (n_species * batch, q_s, q_t), species major; d is a tensor of the
    n_species diffusion coefficients shared by the batch.  The problem must
    have been built with imex=True (it provides op, prec, mass and stiff)."""

    @staticmethod
    def forward(ctx, state0, d, problem, tau, nsteps, kinetics=mf.KIN_NONE, kin=None, tol=1e-10, maxit=200,
                flags=0, checkpoint=50):
        dl = [float(x) for x in d]
        ns = len(dl)
        if state0.shape[0] % ns:
            raise ValueError("state0's leading dimension must be n_species * batch")
        batch = state0.shape[0] // ns
        stepper = mf.Imex(problem.op, problem.prec, problem.mass, tau, dl, kinetics=kinetics, kin=kin, tol=tol,
                          maxit=maxit, flags=flags)
        ws = stepper.workspace(batch, state0.device)
        st = state0.detach().contiguous().clone()
        ckpts = [st.clone()]
        for n in range(nsteps):
            stepper.step(st, batch, workspace=ws)
            if (n + 1) % checkpoint == 0 and n + 1 < nsteps:
                ckpts.append(st.clone())
        ctx.problem, ctx.stepper, ctx.ws, ctx.ckpts = problem, stepper, ws, ckpts
        ctx.nsteps, ctx.checkpoint, ctx.batch, ctx.ns = nsteps, checkpoint, batch, ns
        return st

    @staticmethod
    def backward(ctx, g):
        P, stepper, batch, ns = ctx.problem, ctx.stepper, ctx.batch, ctx.ns
        lam = g.contiguous().clone()
        grad_items = torch.zeros(ns * batch, dtype=torch.float64, device=lam.device)
        aws = stepper.adjoint_workspace(batch, lam.device)
        C, N = ctx.checkpoint, ctx.nsteps
        for k in range(len(ctx.ckpts) - 1, -1, -1):
            s0, s1 = k * C, min(k * C + C, N)
            if s1 <= s0:
                continue
            st = ctx.ckpts[k].clone()
            states = [st.clone()]
            for _ in range(s0, s1 - 1):
                stepper.step(st, batch, workspace=ctx.ws)
                states.append(st.clone())
            # the segment's last output state: recomputed too (the next
            # checkpoint, or the rollout's result)
            stepper.step(st, batch, workspace=ctx.ws)
            states.append(st)
            for j in range(s1 - s0 - 1, -1, -1):
                stepper.adjoint_step(P.stiff, states[j], states[j + 1], lam, grad_items, batch, workspace=aws)
            del states
        dd = None
        if ctx.needs_input_grad[1]:
            dd = torch.zeros(ns, dtype=torch.float64, device=lam.device)
            ones = torch.ones(ns, batch, dtype=torch.float64, device=lam.device)
            # sum over the batch of each species' per-item gradients
            mf.dot_accumulate(grad_items.reshape(ns, batch), ones, dd)
        return lam, dd, None, None, None, None, None, None, None, None, None
