"""The near-contact rule of the GPU parity tests, checked on hand-made traces
(no GPU): a difference is excused only when the first differing trial of each
cell of the earliest differing phase was decided near contact, and every later
difference lies in the light cone of those cells."""
import numpy as np

from oracle.pyoracle import RECORD_DTYPE
from parity_util import near_contact_explains

N_AXIS = 6


def _cell(x, y, z):
    return x + N_AXIS * (y + N_AXIS * z)


def _trace():
    """two trials in each of 8 cells, one cell per phase, in phase order"""
    cells = [_cell(0, 0, 0), _cell(1, 0, 0), _cell(2, 0, 0), _cell(3, 0, 0),
             _cell(4, 0, 0), _cell(0, 3, 0), _cell(0, 0, 3), _cell(3, 3, 3)]
    tr = np.zeros(16, dtype=RECORD_DTYPE)
    for i in range(16):
        tr[i]["cell"] = cells[i // 2]
        tr[i]["phase"] = i // 2
        tr[i]["t"] = i % 2
        tr[i]["particle"] = i
    return tr


def test_identical_traces_pass():
    a = _trace()
    assert near_contact_explains(a, a.copy(), N_AXIS) is None


def test_near_contact_seed_and_its_cell_pass():
    a, b = _trace(), _trace()
    a[0]["near_contact"] = 1
    b[0]["reason"] = 2  # the near-contact trial itself
    b[1]["reason"] = 3  # a later trial of the same cell
    assert near_contact_explains(a, b, N_AXIS) is None


def test_first_difference_must_be_near_contact():
    a, b = _trace(), _trace()
    a[1]["near_contact"] = 1
    b[0]["reason"] = 2  # differs before the near-contact trial
    b[1]["reason"] = 2
    assert "not decided near contact" in near_contact_explains(a, b, N_AXIS)


def test_later_difference_inside_the_light_cone_passes():
    a, b = _trace(), _trace()
    b[0]["near_contact"] = 1
    b[0]["reason"] = 2
    b[4]["reason"] = 1  # cell (2,0,0): distance 2, two phases later
    b[6]["reason"] = 1  # cell (3,0,0): distance 3, three phases later
    assert near_contact_explains(a, b, N_AXIS) is None


def test_later_difference_outside_the_light_cone_fails():
    a, b = _trace(), _trace()
    b[0]["near_contact"] = 1
    b[0]["reason"] = 2
    b[2]["reason"] = 1  # cell (1,0,0), distance 1, one phase later: fine
    b[14]["reason"] = 1  # cell (3,3,3), distance 3, seven phases later: fine
    assert near_contact_explains(a, b, N_AXIS) is None
    c = _trace()
    c[0]["near_contact"] = 1
    c[0]["reason"] = 2
    c[8]["reason"] = 1  # cell (4,0,0): periodic distance 2 at four phases later: fine
    assert near_contact_explains(a, c, N_AXIS) is None
    d = _trace()
    d[2]["near_contact"] = 1  # seed in phase 1, cell (1,0,0)
    d[2]["reason"] = 2
    d[10]["reason"] = 1  # cell (0,3,0): distance 3 at four phases later: fine
    d[6]["reason"] = 1  # cell (3,0,0): distance 2 at two phases later: fine
    assert near_contact_explains(a, d, N_AXIS) is None
    e = _trace()
    e[6]["near_contact"] = 1  # seed in phase 3, cell (3,0,0)
    e[6]["reason"] = 2
    e[10]["reason"] = 1  # cell (0,3,0): distance 3 after two phases: outside
    assert "outside the light cone" in near_contact_explains(a, e, N_AXIS)


def test_unrelated_difference_in_the_seed_phase_fails():
    a, b = _trace(), _trace()
    # two cells of one phase: one near-contact, one not
    for tr in (a, b):
        tr[2]["phase"] = tr[3]["phase"] = 0
    b[0]["near_contact"] = 1
    b[0]["reason"] = 2
    b[2]["reason"] = 1
    assert "not decided near contact" in near_contact_explains(a, b, N_AXIS)


def test_state_difference_without_a_differing_trial_fails():
    a = _trace()
    pa = np.zeros((3, 16))
    pb = pa.copy()
    pb[0, 5] = 1.0
    assert near_contact_explains(a, a.copy(), N_AXIS, pa, pb) is not None
    b = _trace()
    b[0]["near_contact"] = 1
    b[0]["reason"] = 2
    pb2 = pa.copy()
    pb2[1, 0] = 0.5  # particle 0: its trial differs
    assert near_contact_explains(a, b, N_AXIS, pa, pb2) is None
    pb2[1, 9] = 0.5  # particle 9: none of its trials differ
    assert "none of their trials differ" in near_contact_explains(a, b, N_AXIS, pa, pb2)
