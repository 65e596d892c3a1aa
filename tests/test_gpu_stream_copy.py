"""rc_stream_copy (the streaming ceiling the benchmark reports beside the
correction): every launch shape copies exactly, including a partial last
block and a tail of fewer than 16 bytes, and writes nothing past the end."""
import itertools

import numpy as np
import pytest
import torch

import paper_1505_05655_amd as rc
from gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096, 1 << 20, (3 << 20) + 4096 * 7 + 16 * 5 + 9, 17])
def test_copy_shapes(nbytes):
    pad = 4096
    src = torch.randint(-128, 127, (nbytes + 2 * pad,), dtype=torch.int8, device=dev())
    for threads, unroll, policy, wgs in itertools.product((256, 512, 1024), (2, 4, 8), (0, 1, 2),
                                                          (1, 2, 8)):
        if threads * wgs > 2048 or (threads + unroll + policy + wgs) % 3:
            continue
        dst = torch.full((nbytes + 2 * pad,), 7, dtype=torch.int8, device=dev())
        plan = rc.CopyPlan(threads=threads, unroll=unroll, policy=policy, wgs_per_cu=wgs)
        rc.rc_stream_copy(src[pad:], dst[pad:], nbytes, plan)
        torch.cuda.synchronize()
        got = dst.cpu().numpy()
        assert np.array_equal(got[pad:pad + nbytes], src.cpu().numpy()[pad:pad + nbytes]), plan.as_dict()
        assert (got[:pad] == 7).all() and (got[pad + nbytes:] == 7).all(), "write outside"
    # default plan
    dst = torch.zeros_like(src)
    rc.rc_stream_copy(src, dst, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])


def test_copy_rejects():
    a = torch.zeros(4096, dtype=torch.int8, device=dev())
    b = torch.zeros(4096, dtype=torch.int8, device=dev())
    for args in ((a[1:], b, 64, None), (a, a[16:], 64, None),
                 (a, b, 64, rc.CopyPlan(threads=128, unroll=4, policy=0, wgs_per_cu=1)),
                 (a, b, 64, rc.CopyPlan(threads=1024, unroll=4, policy=0, wgs_per_cu=4)),
                 (a, b, 64, rc.CopyPlan(threads=256, unroll=3, policy=0, wgs_per_cu=1)),
                 (a, b, 64, rc.CopyPlan(threads=256, unroll=4, policy=3, wgs_per_cu=1))):
        with pytest.raises(rc.RcError) as e:
            rc.rc_stream_copy(*args)
        assert e.value.status == rc.RC_EINVAL
