"""dns_rhs_noalloc (the context-free right-hand side whose work space is a
file-scope device array) against dns_rhs of a context, through the C ABI:
identical bits on two calls in a row, the second with a smaller grid, in
FP64 and FP32, and a size beyond its scratch refused with an error."""
import numpy as np
import pytest

from gpu_util import note, to_dev
from oracle import ic

pytestmark = pytest.mark.gpu


def _ctx_rhs(uh, N, nu, dtype, dealias):
    from paper_1602_03638_amd import Solver
    s = Solver(N, nu, 1e-3, dtype=dtype, dealias=dealias)
    r = s.set_spectral(uh).rhs()
    s.close()
    return r


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rhs_noalloc_matches_context_rhs(dtype):
    import torch
    import paper_1602_03638_amd as dns
    for N, seed, dealias in ((64, 901, "text"), (32, 902, "appendix")):
        note(f"rhs_noalloc N={N} {dtype} {dealias}")
        h = ic.random_isotropic(N, seed, k0=3.0)
        h = h + 0.05 * np.abs(h).max() * np.random.default_rng(seed).standard_normal(h.shape)
        uh = to_dev(h, dtype)
        got = dns.rhs_noalloc(uh, 0.0137, dealias)
        torch.cuda.synchronize()
        want = _ctx_rhs(uh, N, 0.0137, dtype, dealias)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (N, dtype)


def test_rhs_noalloc_refuses_large_grid():
    import torch
    import paper_1602_03638_amd as dns
    note("rhs_noalloc N=128 refused")
    uh = torch.zeros((3, 128, 128, 65), dtype=torch.complex128, device="cuda")
    with pytest.raises(dns.DnsError) as e:
        dns.rhs_noalloc(uh, 0.01)
    assert e.value.status == dns.DNS_E_INVAL and "N <= 64" in str(e.value)
