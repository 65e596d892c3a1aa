"""Bilinear Bayer demosaicing on the GPU (rc_demosaic) against the CPU oracle,
bit-exact (integer averages): hand-worked images, ragged shapes around the
256-column wave width and the row-band height, full-scale samples, the
paper's 2048 x 2048 image and a batch of them, with guard bands around the
output."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_1505_05655_amd as rc
import pins_demosaic

pytestmark = pytest.mark.gpu

SENTINEL = 0x5A5A


def dev():
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def o():
    return oracle.get()


def gpu_demosaic(raw):
    I, H, W = raw.shape
    n = I * 3 * H * W
    buf = torch.full((n + 64,), SENTINEL, dtype=torch.int16, device=dev())
    out = buf[32:32 + n].view(I, 3, H, W)
    rc.demosaic(torch.from_numpy(raw.view(np.int16)).to(dev()), out=out)
    torch.cuda.synchronize()
    host = buf.cpu().numpy()
    assert np.all(host[:32] == SENTINEL) and np.all(host[32 + n:] == SENTINEL), "guard band"
    return out.cpu().numpy().view(np.uint16)


def test_hand_worked_images(o):
    for name, img in pins_demosaic.IMAGES.items():
        raw = np.ascontiguousarray(img[None])
        assert np.array_equal(gpu_demosaic(raw), o.demosaic(raw)), name


SHAPES = [(1, 2, 4), (1, 2, 8), (2, 6, 12), (1, 4, 256), (1, 10, 260), (1, 64, 512),
          (3, 130, 1028), (2, 66, 4), (1, 200, 1024)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_random_mosaics(o, shape):
    rng = np.random.default_rng(sum(shape))
    raw = rng.integers(0, 65536, shape).astype(np.uint16)
    assert np.array_equal(gpu_demosaic(raw), o.demosaic(raw))


def test_full_scale_and_zero(o):
    for v in (0, 65535):
        raw = np.full((1, 8, 16), v, np.uint16)
        assert np.array_equal(gpu_demosaic(raw), o.demosaic(raw))


@pytest.mark.parametrize("w", [0, 1])
def test_demosaic_workloads(o, w):
    name, seed, cfg, images, H, W = gen.demosaic_workload(w)
    raw = gen.bayer(seed, cfg, 0, images, H, W)
    assert np.array_equal(gpu_demosaic(raw), o.demosaic(raw)), name


def test_rejects_bad_shapes():
    raw = torch.zeros((1, 4, 6), dtype=torch.int16, device=dev())
    with pytest.raises(rc.RcError) as e:
        rc.demosaic(raw)  # width not a multiple of 4
    assert e.value.status == rc.RC_EINVAL
    raw = torch.zeros((1, 3, 8), dtype=torch.int16, device=dev())
    with pytest.raises(rc.RcError):
        rc.demosaic(raw)  # odd height
