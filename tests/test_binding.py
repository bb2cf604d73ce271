"""Host-side checks of the Python binding (no GPU): what it hands to the C ABI
as a raw pointer must hold the tensor's values in memory."""
import pytest
import torch

from paper_2004_11346_amd.sht import check_tensor, materialize


def test_lazy_conj_and_neg_views_are_rejected():
    x = torch.randn(2, 3, dtype=torch.complex128)
    check_tensor(x, torch.complex128, (2, 3), "x", require_cuda=False)
    for bad in (x.conj(), torch._neg_view(x), x.conj().t().t()):
        assert bad.is_conj() or bad.is_neg()
        with pytest.raises(ValueError):
            check_tensor(bad, torch.complex128, (2, 3), "x", require_cuda=False)
    with pytest.raises(ValueError):
        check_tensor(x.t(), torch.complex128, (3, 2), "x", require_cuda=False)
    with pytest.raises(TypeError):
        check_tensor(x, torch.complex64, (2, 3), "x", require_cuda=False)
    with pytest.raises(TypeError):
        check_tensor(x, torch.complex128, (2, 3), "x")  # host tensor where a device one is needed


def test_materialize_resolves_lazy_views():
    x = torch.randn(4, 5, dtype=torch.complex128)
    for v, ref in ((x.conj(), torch.conj_physical(x)), (torch._neg_view(x), -x), (x.conj().t(), torch.conj_physical(x).t())):
        m = materialize(v)
        assert not m.is_conj() and not m.is_neg() and m.is_contiguous()
        assert torch.equal(m, ref.contiguous())
        # the raw memory is what the C ABI reads
        raw = torch.view_as_real(m).flatten()
        assert torch.equal(raw, torch.view_as_real(ref.contiguous()).flatten())


def test_autograd_gradient_of_a_conjugated_output_is_resolved():
    """The backward receives grad_f with the conjugate bit set when the loss
    reaches f only through f.conj(); the function must resolve it before
    handing memory to the adjoint kernel."""
    seen = {}

    class Probe(torch.autograd.Function):
        @staticmethod
        def forward(ctx, b):
            return b.clone()

        @staticmethod
        def backward(ctx, g):
            seen["raw_conj"] = g.is_conj()
            m = materialize(g)
            seen["resolved_conj"] = m.is_conj()
            return m

    b = torch.randn(3, dtype=torch.complex128, requires_grad=True)
    f = Probe.apply(b)
    w = torch.randn(3, dtype=torch.complex128)
    (f.conj() * w).real.sum().backward()
    assert seen["resolved_conj"] is False
    # gradient of Re(sum conj(f) w) w.r.t. b in torch's convention is conj(conj(w)) = w
    assert torch.allclose(b.grad, w)
