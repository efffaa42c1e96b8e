"""Host emulation of the face-flux array addressing shared by the flux kernel
(writer) and the cell update (reader), transcribed from their index
arithmetic: F_d holds n_d + 1 faces along a wall normal and n_d along a
periodic one (face n is face 0), rows padded to 32 elements.  Every cell's
two faces of every direction address slots the flux kernel writes, the left
slot holds the cell's left face and the right slot its right face, which on
a periodic axis is face 0 for the last cell.  The same arithmetic with n
faces on a periodic normal axis and the last face stored as a copy of the
first in slot n (a variant that was measured wrong on y faces and reverted)
puts the copy of a y-face row onto the first row of the next z plane: the
aliasing that explains the wrong y-face fluxes."""
import itertools

import numpy as np


def pitch(n):
    return (n + 31) & ~31


def face_index(fe, f):
    return ((f[2] * fe[1]) + f[1]) * pitch(fe[0]) + f[0]


def written_slots(n, d, nfaces_normal):
    fe = list(n)
    fe[d] = nfaces_normal
    return fe, {face_index(fe, f): f for f in itertools.product(*(range(e) for e in fe))}


def update_slots(n, d, fe, i, j, k, wrap=True):
    """The update's left and right face slots of cell (i, j, k) for direction d
    (a periodic normal holds n faces: the last cell's right face is face 0;
    wrap=False: the reverted variant's read of slot n)."""
    fm = ((k * fe[1] + j) * pitch(fe[0])) + i
    step = 1 if d == 0 else (pitch(fe[0]) if d == 1 else pitch(fe[0]) * fe[1])
    c = (i, j, k)[d]
    fp = fm - c * step if wrap and fe[d] == n[d] and c == n[d] - 1 else fm + step
    return fm, fp


def test_update_reads_the_faces_the_flux_kernel_writes():
    for n in [(4, 5, 6), (33, 8, 12), (32, 32, 7), (20, 16, 12)]:
        for d in range(3):
            for periodic in (True, False):
                fe, slots = written_slots(n, d, n[d] if periodic else n[d] + 1)
                for i, j, k in itertools.product(range(n[0]), range(n[1]), range(n[2])):
                    fm, fp = update_slots(n, d, fe, i, j, k)
                    c = [i, j, k]
                    right = list(c)
                    right[d] += 1
                    if periodic:
                        right[d] %= n[d]
                    assert slots[fm] == tuple(c) and slots[fp] == tuple(right), (n, d, periodic, c)


def test_n_face_variant_aliases_the_next_plane():
    n = (20, 16, 12)
    fe, slots = written_slots(n, 1, n[1])  # n faces along y
    # the copy of face 0 of row (i, k), stored at the flat slot of face n
    i, k = 3, 4
    copy_slot = face_index(fe, (i, n[1], k))
    assert slots[copy_slot] == (i, 0, k + 1)  # a real face of the next z plane
    # and the update of cell j = n - 1 reads that slot as its right face
    _, fp = update_slots(n, 1, fe, i, n[1] - 1, k, wrap=False)
    assert fp == copy_slot
