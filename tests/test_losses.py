"""Host-side checks of the training losses (Sec. 4.2, 4.3; Eq. 6, 7): the
package has no CPU implementation of them; the CPU references are the
oracle's (oracle/ssim.py, oracle/regularisers.py), pinned in
test_oracle_ssim.py and test_oracle_reg.py."""
import pytest
import torch

from paper_2504_17954_amd import inputs as I
from paper_2504_17954_amd import losses as L


def test_ssim_refuses_host_tensors():
    x = torch.rand((4, 20, 24))
    with pytest.raises(ValueError):
        L.ssim(x, x)
    with pytest.raises(ValueError):
        L.photometric(x, x)


def test_regularisers_refuse_host_tensors():
    cam = I.look_at((0.0, -3.0, 0.0), width=24, height=20)
    depth, alpha = torch.ones((20, 24)), torch.ones((20, 24))
    with pytest.raises(ValueError):
        L.regularisers(depth, alpha, cam, normal=torch.ones((3, 20, 24)))
