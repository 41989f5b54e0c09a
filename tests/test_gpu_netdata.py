"""GPU checks of the training-set preparation kernels (lesnet_crop,
lesnet_gather, lesnet_sum_squares, lesnet_scale_div) through the C ABI
against numpy on the host: windows and their y-mirror images and gathers
bit for bit, the float64 sum of squares to rounding, the float32 division
bit for bit."""
import numpy as np
import pytest

import paper_1504_02264_amd as les

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("mirror", [False, True])
@pytest.mark.parametrize("shape,window", [((20, 24, 36, 3), (4, 8, 12, 8, 12, 16)),
                                          ((9, 7, 5, 3), (0, 0, 0, 9, 7, 5)),
                                          ((12, 16, 8), (5, 3, 1, 4, 13, 7))])
def test_crop_and_mirror(shape, window, mirror):
    import torch
    rng = np.random.default_rng(sum(shape) + 7 * mirror)
    a = rng.standard_normal(shape).astype(np.float32)
    got = les.crop(_dev(a), window, mirror_y=mirror)
    torch.cuda.synchronize()
    z, y, x, cd, ch, cw = window
    ref = a[z:z + cd, y:y + ch, x:x + cw]
    if mirror:
        ref = ref[:, ::-1]
    assert np.array_equal(got.cpu().numpy(), ref)


def test_gather_items():
    import torch
    rng = np.random.default_rng(3)
    a = rng.standard_normal((11, 4, 6, 5, 3)).astype(np.float32)
    idx = np.array([7, 0, 10, 3, 3], np.int32)
    got = les.gather(_dev(a), idx)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), a[idx])


def test_sum_squares_and_scale():
    import torch
    rng = np.random.default_rng(5)
    a = (rng.standard_normal(3_000_017) * 3.0).astype(np.float32)
    s = les.sum_squares(_dev(a))
    ref = float(np.sum(a.astype(np.float64) ** 2))
    assert s == pytest.approx(ref, rel=1e-13)
    assert les.sum_squares(_dev(np.zeros(0, np.float32))) == 0.0
    scale = float(np.sqrt(ref / a.size))
    got = les.scale_div(_dev(a), scale)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), a / np.float32(scale))


def test_data_prep_rejects_bad_arguments():
    import torch
    a = _dev(np.zeros((4, 4, 4, 3), np.float32))
    with pytest.raises(les.LesError):
        les.crop(a, (1, 0, 0, 4, 4, 4))          # window past the end
    with pytest.raises(les.LesError):
        les.gather(a, np.array([4], np.int32))   # index past the end
    with pytest.raises(les.LesError):
        les.gather(a, np.zeros(65, np.int32))    # more than 64 items
    with pytest.raises(les.LesError):
        les.scale_div(a, 0.0)
    torch.cuda.synchronize()


def test_mirror_y_pairs():
    """warmstart.mirror_y: the pairs, then their mirror images in y, in the
    library's kernels."""
    import torch
    from paper_1504_02264_amd import warmstart as ws
    X = torch.arange(2 * 4 * 6 * 8 * 3, dtype=torch.float32).reshape(2, 4, 6, 8, 3).cuda()
    T = torch.arange(2 * 4 * 6 * 8, dtype=torch.float32).reshape(2, 4, 6, 8).cuda()
    Xm, Tm = ws.mirror_y(X, T)
    torch.cuda.synchronize()
    assert Xm.shape == (4, 4, 6, 8, 3) and Tm.shape == (4, 4, 6, 8)
    assert torch.equal(Xm[:2], X) and torch.equal(Tm[:2], T)
    assert torch.equal(Xm[3, 1, 0, 2], X[1, 1, 5, 2]) and torch.equal(Tm[2, 3, 1, 7], T[0, 3, 4, 7])
    assert Xm.is_contiguous() and Tm.is_contiguous()
