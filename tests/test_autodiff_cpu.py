"""Host-side pieces of the differentiable TDVP layer (no device needed)."""
import torch


def test_projection_backward_matches_gradcheck():
    """Custom backward of one Gram-Schmidt pass against finite differences."""
    from paper_1912_06127_amd.autodiff import Project
    g = torch.Generator().manual_seed(5)
    n, k = 7, 3
    V = [torch.randn(n, dtype=torch.complex128, generator=g, requires_grad=True) for _ in range(k)]
    w = torch.randn(n, dtype=torch.complex128, generator=g, requires_grad=True)
    assert torch.autograd.gradcheck(lambda w_, *V_: Project.apply(w_, *V_), (w, *V), eps=1e-6, atol=1e-8)


def test_projection_forward_is_one_gram_schmidt_pass():
    from paper_1912_06127_amd.autodiff import Project
    g = torch.Generator().manual_seed(6)
    Q, _ = torch.linalg.qr(torch.randn(9, 4, dtype=torch.complex128, generator=g))
    w = torch.randn(9, dtype=torch.complex128, generator=g)
    out = Project.apply(w, *Q.T)
    assert torch.allclose(Q.conj().T @ out, torch.zeros(4, dtype=torch.complex128), atol=1e-14)
    assert torch.allclose(out, w - Q @ (Q.conj().T @ w), atol=1e-14)
