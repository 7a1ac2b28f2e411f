"""The streaming copy kernel that measures achievable bandwidth (the paper's
b_S in its roofline estimate, Sec. 4.3) moves exactly the bytes it is given:
bit-exact copies for one element, a ragged grid tail and a large buffer, and
nothing written past the end."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, (1 << 20) + 48, 64 << 20])
def test_copy_probe_is_an_exact_copy(nbytes):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2402_13171_amd.lbm import copy_probe
    print(f"copy probe: {nbytes} bytes", flush=True)
    g = torch.Generator().manual_seed(nbytes % 1000003)
    src_h = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g)
    src = src_h.to("cuda")
    tail = 4096
    dst = torch.full((nbytes + tail,), 0xA5, dtype=torch.uint8, device="cuda")
    copy_probe(src, dst[:nbytes])
    torch.cuda.synchronize()
    out = dst.cpu().numpy()
    assert np.array_equal(out[:nbytes], src_h.numpy())
    assert np.all(out[nbytes:] == 0xA5)


def test_copy_probe_binding_rejects_strided_and_mismatched_views():
    """The kernel copies numel * element_size bytes from the base pointers, so
    the binding refuses views that do not cover that range contiguously."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2402_13171_amd.lbm import copy_probe
    a = torch.zeros((64, 64), device="cuda")
    b = torch.zeros((64, 64), device="cuda")
    with pytest.raises(ValueError, match="not contiguous"):
        copy_probe(a.t(), b)
    with pytest.raises(ValueError, match="not contiguous"):
        copy_probe(a, b[:, ::2].repeat(1, 2)[:, ::2].t())
    with pytest.raises(ValueError, match="differ in size"):
        copy_probe(a, b[:32])
    with pytest.raises(ValueError, match="not a device tensor"):
        copy_probe(a, torch.zeros((64, 64)))
