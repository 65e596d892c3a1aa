"""Gradient-based (adaptive colour plane) Bayer demosaicing on the GPU
(rc_demosaic_gradient) against the CPU oracle, bit-exact (integer
arithmetic): hand-worked images, random and smooth mosaics (smooth ones make
ties and unclamped estimates common) in ragged shapes around the 256-column
wave width, the wave edges where the edge lanes compute the green beyond the
wave, and the row bands whose halos are recomputed; step edges, full-scale
samples, the paper's 2048 x 2048 image and a batch of 16, with guard bands
around the output."""
import numpy as np
import pytest
import torch
from scipy import ndimage

import gen
import oracle
import paper_1505_05655_amd as rc
import pins_demosaic_gradient

pytestmark = pytest.mark.gpu

SENTINEL = 0x5A5A


def dev():
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def o():
    return oracle.get()


def gpu_gradient(raw):
    I, H, W = raw.shape
    n = I * 3 * H * W
    buf = torch.full((n + 64,), SENTINEL, dtype=torch.int16, device=dev())
    out = buf[32:32 + n].view(I, 3, H, W)
    rc.demosaic(torch.from_numpy(raw.view(np.int16)).to(dev()), out=out, method="gradient")
    torch.cuda.synchronize()
    host = buf.cpu().numpy()
    assert np.all(host[:32] == SENTINEL) and np.all(host[32 + n:] == SENTINEL), "guard band"
    return out.cpu().numpy().view(np.uint16)


def smooth(rng, shape):
    noise = rng.integers(0, 65536, shape).astype(np.float64)
    return (ndimage.uniform_filter(noise, (1, 5, 5)) / 4).astype(np.uint16)


def test_hand_worked_images(o):
    for name, img in pins_demosaic_gradient.IMAGES.items():
        raw = np.array(img, dtype=np.uint16)[None]
        assert np.array_equal(gpu_gradient(raw), o.demosaic_gradient(raw)), name


SHAPES = [(1, 4, 4), (1, 4, 8), (2, 6, 12), (1, 4, 256), (1, 10, 260), (1, 64, 512),
          (3, 130, 1028), (2, 66, 4), (1, 200, 1024), (1, 34, 2048), (5, 18, 516),
          (1, 4, 1020), (1, 20, 8192)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_random_and_smooth_mosaics(o, shape):
    rng = np.random.default_rng(sum(shape) + 7)
    raw = rng.integers(0, 65536, shape).astype(np.uint16)
    assert np.array_equal(gpu_gradient(raw), o.demosaic_gradient(raw)), "random"
    raw = smooth(rng, shape)
    assert np.array_equal(gpu_gradient(raw), o.demosaic_gradient(raw)), "smooth"


def test_edges_full_scale_and_zero(o):
    H, W = 36, 520  # steps at the wave boundary (column 256) and a band boundary (row 16)
    cols, rows = np.arange(W)[None, :] * np.ones((H, 1)), np.arange(H)[:, None] * np.ones((1, W))
    for k in (255, 256, 257, 258):
        raw = np.where(cols < k, 1000, 3000).astype(np.uint16)[None]
        assert np.array_equal(gpu_gradient(raw), o.demosaic_gradient(raw)), ("column", k)
    for k in (15, 16, 17, 18):
        raw = np.where(rows < k, 1000, 3000).astype(np.uint16)[None]
        assert np.array_equal(gpu_gradient(raw), o.demosaic_gradient(raw)), ("row", k)
    for v in (0, 65535):
        raw = np.full((1, 8, 16), v, np.uint16)
        assert np.array_equal(gpu_gradient(raw), o.demosaic_gradient(raw))
    checker = ((np.indices((8, 260)).sum(0) % 2) * 65535).astype(np.uint16)[None]
    assert np.array_equal(gpu_gradient(checker), o.demosaic_gradient(checker))


# Launches of at least 8 waves per CU with whole groups of 4 column waves
# pass the green values beyond each wave through LDS; these take that path,
# one with a last band of 2 rows, one whose last wave is short of a lane.
LARGE = [(16, 512, 1024), (2, 2048, 4096), (16, 522, 1024), (16, 512, 1020)]


@pytest.mark.parametrize("shape", LARGE, ids=lambda s: "x".join(map(str, s)))
def test_large_launches(o, shape):
    rng = np.random.default_rng(sum(shape) + 11)
    raw = smooth(rng, shape)
    raw[:, ::7, ::5] = rng.integers(0, 65536, raw[:, ::7, ::5].shape)
    assert np.array_equal(gpu_gradient(raw), o.demosaic_gradient(raw))


@pytest.mark.parametrize("w", [0, 1])
def test_demosaic_workloads(o, w):
    name, seed, cfg, images, H, W = gen.demosaic_workload(w)
    raw = gen.bayer(seed, cfg, 0, images, H, W)
    assert np.array_equal(gpu_gradient(raw), o.demosaic_gradient(raw)), name


def test_rejects_bad_shapes():
    for shape in ((1, 4, 6), (1, 3, 8), (1, 2, 8)):  # width % 4, odd height, height 2
        raw = torch.zeros(shape, dtype=torch.int16, device=dev())
        with pytest.raises(rc.RcError) as e:
            rc.demosaic(raw, method="gradient")
        assert e.value.status == rc.RC_EINVAL
