"""Quadrant check (mtb_align_quadrants) against the oracle: per-quadrant shifts,
level-0 errors and the rotation flag, bit-exact."""

import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import _rotate_nearest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def mtb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_06483_amd as m

    m.lib()
    return m


def _dev(img, extra=0):
    h, w, _ = img.shape
    buf = torch.zeros((h, w + extra, 3), dtype=torch.uint8, device=DEV)
    buf[:, :w] = torch.from_numpy(np.ascontiguousarray(img)).to(DEV)
    return buf[:, :w]


def _check(mtb, ref, mov, L, tol=1, extra=0):
    want = oracle.align_quadrants(ref, mov, L, tolerance=tol)
    got = mtb.mtb_align_quadrants(_dev(ref, extra), _dev(mov, extra), L, tolerance=tol)
    torch.cuda.synchronize()
    assert np.array_equal(got["shifts"].cpu().numpy(), want["shifts"])
    assert np.array_equal(got["errs"].cpu().numpy().astype(np.int64), want["errs"])
    assert int(got["flag"].cpu()[0]) == want["flag"]
    return want


@pytest.mark.parametrize("w,h,extra", [(480, 360, 0), (481, 363, 0), (641, 479, 5)])
def test_quadrants_translation(mtb, w, h, extra):
    base = synth.expose(synth.rect_field(w, h, 60, np.random.default_rng(w)), 0.0)
    want = _check(mtb, base, synth.translate(base, 4, -6), 5, extra=extra)
    assert want["flag"] == 0


@pytest.mark.parametrize("deg,tol", [(3.0, 1), (3.0, 40), (-2.0, 1)])
def test_quadrants_rotation(mtb, deg, tol):
    base = synth.expose(synth.rect_field(480, 360, 60, np.random.default_rng(43)), 0.0)
    want = _check(mtb, base, _rotate_nearest(base, deg), 5, tol=tol)
    assert want["flag"] == (1 if tol == 1 else 0)


def test_quadrants_blob_exposures(mtb):
    ref, mov, _ = synth.make_pair(800, 600, 120, 44, 20)
    _check(mtb, ref, mov, 6)
