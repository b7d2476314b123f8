"""The ground-truth IoU measure (the analogue of Table I's plane IoU): exact
values for congruent, half-overlapping, disjoint and rotated polygons, the
normal and offset gates, and the best match over several planes."""
import numpy as np

import scenes


def _rect():
    return scenes.Rect((1.0, 2.0, 0.5), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.4, 0.2)


def _poly(uv, z=0.5, c=(1.0, 2.0)):
    uv = np.asarray(uv, np.float64)
    return np.c_[uv[:, 0] + c[0], uv[:, 1] + c[1], np.full(len(uv), z)]


def test_exact_values():
    r = _rect()
    same = _poly([[-0.4, -0.2], [0.4, -0.2], [0.4, 0.2], [-0.4, 0.2]])
    assert abs(scenes.polygon_iou_with_rect(r, same) - 1.0) < 1e-12
    assert abs(scenes.polygon_iou_with_rect(r, same[::-1]) - 1.0) < 1e-12      # orientation does not matter
    half = _poly([[0.0, -0.2], [0.8, -0.2], [0.8, 0.2], [0.0, 0.2]])           # shifted by half its width
    assert abs(scenes.polygon_iou_with_rect(r, half) - 1.0 / 3.0) < 1e-12
    far = _poly([[1.0, -0.2], [1.8, -0.2], [1.8, 0.2], [1.0, 0.2]])
    assert scenes.polygon_iou_with_rect(r, far) == 0.0
    # a diamond through the midpoints of the edges: half the rectangle, inside it
    dia = _poly([[0.4, 0.0], [0.0, 0.2], [-0.4, 0.0], [0.0, -0.2]])
    assert abs(scenes.polygon_iou_with_rect(r, dia) - 0.5) < 1e-12
    # a square of side 0.4 rotated 45 degrees about the centre: its corners stick out of the 0.4 m high rectangle
    h = 0.2 * np.sqrt(2.0)
    rot = _poly([[h, 0.0], [0.0, h], [-h, 0.0], [0.0, -h]])
    # inside part: the rotated square minus the two tips above/below |v| <= 0.2 (each a triangle of
    # height h - 0.2 and base 2 (h - 0.2)) -> area 0.16 - 2 (h - 0.2)^2
    inter = 0.16 - 2 * (h - 0.2) ** 2
    assert abs(scenes.polygon_iou_with_rect(r, rot) - inter / (0.32 + 0.16 - inter)) < 1e-12


def test_gates_and_best_match():
    r = _rect()
    same = _poly([[-0.4, -0.2], [0.4, -0.2], [0.4, 0.2], [-0.4, 0.2]])
    half = _poly([[0.0, -0.2], [0.8, -0.2], [0.8, 0.2], [0.0, 0.2]])
    planes = np.array([[0.0, 0.0, 1.0, -0.5], [0.0, 0.0, -1.0, 0.5], [1.0, 0.0, 0.0, -1.0],
                       [0.0, 0.0, 1.0, -0.7], [np.nan, 0, 0, 0]])
    polys = [half, same, same, same, same]
    # plane 0: IoU 1/3; plane 1 (flipped normal) 1; plane 2 wrong normal, plane 3 0.2 m away, plane 4 NaN: gated
    assert abs(scenes.plane_iou([r], planes, polys)[0] - 1.0) < 1e-12
    assert abs(scenes.plane_iou([r], planes[[0, 2, 3, 4]], [half, same, same, same])[0] - 1.0 / 3.0) < 1e-12
    assert scenes.plane_iou([r], planes[[2, 3]], [same, same])[0] == 0.0
