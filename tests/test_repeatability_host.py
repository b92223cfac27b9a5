"""Host logic of the repeatability harness: 3 x 3 non-maximum suppression,
greedy one-to-one matching and F1 on hand-built cases, and the generator's
labels (interior angles, corners moving with the rotation)."""
import numpy as np

from paper_2410_04090_amd import repeatability as R
from synth import corners


def test_nms_keeps_strict_maxima_and_first_of_ties():
    r = np.zeros((7, 7), np.uint16)
    r[2, 2] = 50
    r[2, 3] = 40                      # suppressed by (2, 2)
    r[5, 1] = 30
    r[5, 2] = 30                      # equal neighbour later in raster order: suppressed
    r[0, 6] = 10                      # isolated, on the border
    ys, xs = R.nms3(r)
    assert sorted(zip(ys.tolist(), xs.tolist())) == [(0, 6), (2, 2), (5, 1)]
    assert len(R.nms3(np.zeros((4, 4), np.uint16))[0]) == 0


def test_match_f1_cases():
    gt = np.array([[10.0, 10.0], [20.0, 10.0], [30.0, 30.0]])
    m = R.match_f1(gt.copy(), gt, 3.0)
    assert (m["tp"], m["f1"]) == (3, 1.0)
    m = R.match_f1(np.zeros((0, 2)), gt, 3.0)
    assert (m["tp"], m["precision"], m["recall"], m["f1"]) == (0, 0.0, 0.0, 0.0)
    # two detections near one corner: one pair only (one to one)
    det = np.array([[10.5, 10.0], [11.0, 10.0], [50.0, 50.0]])
    m = R.match_f1(det, gt, 3.0)
    assert m["tp"] == 1 and abs(m["precision"] - 1 / 3) < 1e-12 and abs(m["recall"] - 1 / 3) < 1e-12
    # the closer pair wins: detection 0 takes corner 1, detection 1 is left over
    det = np.array([[18.5, 10.0], [19.0, 10.0]])
    g2 = np.array([[16.0, 10.0], [19.0, 10.0]])
    m = R.match_f1(det, g2, 3.0)
    assert m["tp"] == 2                # 1-1 at distance 0, then 0-0 at 2.5
    # beyond the tolerance: no pair
    assert R.match_f1(np.array([[14.0, 10.0]]), gt, 3.0)["tp"] == 0
    assert R.match_f1(np.array([[13.0, 10.0]]), gt, 3.0)["tp"] == 1


def test_interior_angles_and_rotated_labels():
    sq = (np.array([0.0, 10, 10, 0]), np.array([0.0, 0, 10, 10]))
    assert np.allclose(corners.interior_angles(*sq), 90.0)
    arrow = (np.array([0.0, 10, 5, 10, 0]), np.array([0.0, 0, 5, 10, 10]))
    assert np.allclose(corners.interior_angles(*arrow), [90, 45, 270, 45, 90])
    sc = corners.corner_scene(3)
    _, g0 = corners.render_rotated(sc, 0, [3, 1])
    _, g90 = corners.render_rotated(sc, 90, [3, 2])
    # a quarter turn about the centre maps the label set onto itself rotated
    c = sc.width / 2.0 - 0.5
    rot = np.stack([c - (g0[:, 1] - c), c + (g0[:, 0] - c)], 1)
    assert len(g0) == len(g90) > 20
    d = np.abs(np.sort(rot, axis=0) - np.sort(g90, axis=0)).max()
    assert d < 1e-6
