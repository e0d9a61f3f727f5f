"""EdgeGrad's forward pass is the identity (supplement, 'EdgeGrad module'):
bit-identical output sharing the input's storage.  Runs on CPU tensors, no
kernel is called in the forward pass."""
import torch

from paper_2405_02508_amd.autograd import EdgeGrad


def test_p12_edgegrad_forward_is_identity():
    g = torch.Generator().manual_seed(0)
    img = torch.randn(37, 5, generator=g, dtype=torch.float32)
    img[3, 2] = float("nan")
    img[4, 1] = -0.0
    v = torch.randn(10, 3, generator=g)
    tid = torch.zeros(37, dtype=torch.int32)
    out = EdgeGrad.apply(img, v, tid, None)
    assert out.data_ptr() == img.data_ptr()
    assert torch.equal(out.view(torch.int32), img.view(torch.int32))
