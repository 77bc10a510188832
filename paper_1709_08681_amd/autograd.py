"""torch.autograd.Function around psc_predict with the hand-written adjoint.

Forward calls psc_predict; backward calls psc_predict_vjp, which rebuilds the
baseline kernels and their offset derivatives (Eq. DA) from the saved offsets
instead of storing them.  With PyTorch's convention for complex tensors the
incoming gradient G of a real loss is dL/dRe(V) + i dL/dIm(V), so
dL/dp_a = sum Re(conj(G) dV/dp_a), which is what psc_predict_vjp returns.
"""
import torch


class PscPredict(torch.autograd.Function):
    @staticmethod
    def forward(ctx, offsets, session):
        if offsets.dtype != torch.float64:
            raise TypeError("offsets must be float64")
        off = offsets.detach().contiguous()
        vis = session.predict(off)
        ctx.session = session
        ctx.save_for_backward(off)
        return vis

    @staticmethod
    def backward(ctx, grad_vis):
        (off,) = ctx.saved_tensors
        g = ctx.session.vjp(off, grad_vis.to(torch.complex64).contiguous())
        return g, None


def predict(offsets, session):
    """Differentiable model visibilities [n_row, n_chan, n_pol] complex64."""
    return PscPredict.apply(offsets, session)
