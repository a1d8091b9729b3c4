"""Host-side checks of the front-zone helper used by the running-point search
(Sec. 5.1: four front-field zones that move with the ball): every zone is a
valid window of the 0.1 m lattice, zones III/IV lie in front of I/II and on
both sides of the long axis, and the zones follow the ball up the field."""
import pytest

from paper_1909_07717_amd.framegen import Params
from paper_1909_07717_amd.zones import front_zones


def _x_range(z, p):
    h, i0, j0, nx, ny = z
    nxa = int(round(p.field_len / float(h))) + 1
    x0 = float(h) * (i0 - (nxa - 1) / 2)
    return x0, x0 + float(h) * (nx - 1)


@pytest.mark.parametrize("bx", [-6.0, -3.0, 0.0, 1.7, 4.0, 6.0])
@pytest.mark.parametrize("by", [-4.5, 0.0, 3.2])
def test_front_zones_are_valid_windows(bx, by):
    p = Params()
    zones = front_zones((bx, by), p)
    assert len(zones) == 4
    nxa, nya = 121, 91
    for h, i0, j0, nx, ny in zones:
        assert float(h) == pytest.approx(0.1)
        assert i0 >= 0 and j0 >= 0 and nx > 0 and ny > 0
        assert i0 + nx <= nxa and j0 + ny <= nya
    # back zones (I, II) end where the front ones (III, IV) start
    xb = [_x_range(z, p) for z in zones]
    assert xb[0] == xb[1] and xb[2] == xb[3]
    assert xb[0][1] == pytest.approx(xb[2][0])
    # each half split at y = 0
    assert zones[0][2] < zones[1][2] and zones[2][2] < zones[3][2]


def test_front_zones_follow_the_ball():
    p = Params()
    starts = [_x_range(front_zones((bx, 0.0), p)[0], p)[0] for bx in (-4.0, -1.0, 1.0, 3.0)]
    assert starts == sorted(starts) and starts[0] < starts[-1]
