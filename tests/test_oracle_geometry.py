"""Pins of the geometry oracle (droplet count and mean radius, Section 4.2.2): Euler
characteristics of shapes with known topology, brute-force component counts of
random sets (scipy.ndimage.label), and Eq. Rmoy_2D on exact tanh droplets."""

import numpy as np
import pytest
from scipy import ndimage

from oracle import geometry

WALLS = ("walls", "walls", "walls")
PER = ("periodic", "periodic", "periodic")


def disk(n, cx, cy, r):
    y, x = np.mgrid[0:n, 0:n]
    return ((x - cx) ** 2 + (y - cy) ** 2 <= r * r).astype(float)[None]


def ball(n, c, r):
    z, y, x = np.mgrid[0:n, 0:n, 0:n]
    return ((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= r * r).astype(float)


def test_elementary_complexes():
    one = np.zeros((1, 5, 5)); one[0, 2, 2] = 1
    assert geometry.euler_characteristic(one, WALLS) == 1
    assert geometry.euler_characteristic(np.ones((1, 6, 7)), PER) == 0          # the 2-torus
    assert geometry.euler_characteristic(np.ones((1, 6, 7)), WALLS) == 1        # a disk
    assert geometry.euler_characteristic(np.ones((4, 5, 6)), PER) == 0          # the 3-torus
    assert geometry.euler_characteristic(np.ones((4, 5, 6)), WALLS) == 1        # a ball
    cube = np.zeros((3, 3, 3)); cube[1, 1, 1] = 1
    assert geometry.euler_characteristic(cube, WALLS) == 1


def test_known_topologies_2d():
    n = 64
    assert geometry.euler_characteristic(disk(n, 20, 30, 8), WALLS) == 1
    assert geometry.euler_characteristic(disk(n, 20, 30, 8) + disk(n, 45, 30, 8), WALLS) == 2
    annulus = disk(n, 32, 32, 20) - disk(n, 32, 32, 10)
    assert geometry.euler_characteristic(annulus, WALLS) == 0
    # a band that wraps around the periodic x axis is an annulus of the torus
    band = np.zeros((1, n, n)); band[0, 20:30, :] = 1
    assert geometry.euler_characteristic(band, PER) == 0
    assert geometry.euler_characteristic(band, ("walls", "periodic", "periodic")) == 1
    # a disk cut by the periodic edge is still one droplet
    assert geometry.euler_characteristic(disk(n, 2, 3, 8) + disk(n, 2 + n, 3, 8) + disk(n, 2, 3 + n, 8)
                                         + disk(n, 2 + n, 3 + n, 8), PER) == 1


def test_known_topologies_3d():
    n = 32
    assert geometry.euler_characteristic(ball(n, (10, 12, 14), 6), WALLS) == 1
    assert geometry.euler_characteristic(ball(n, (8, 8, 8), 5) + ball(n, (22, 22, 22), 5), WALLS) == 2
    shell = ball(n, (16, 16, 16), 12) - ball(n, (16, 16, 16), 7)
    assert geometry.euler_characteristic(shell, WALLS) == 2                     # ball with a cavity
    z, y, x = np.mgrid[0:n, 0:n, 0:n]
    torus = ((np.sqrt((x - 16) ** 2 + (y - 16) ** 2) - 9) ** 2 + (z - 16) ** 2 <= 9).astype(float)
    assert geometry.euler_characteristic(torus, WALLS) == 0                     # solid torus


@pytest.mark.parametrize("seed", range(6))
def test_random_sets_2d_against_labelling(seed):
    """Bounded 2D sets: chi = components (8-connected) - holes (4-connected components
    of the complement that do not reach the edge)."""
    rng = np.random.default_rng(seed)
    a = rng.random((40, 37)) < (0.3 + 0.08 * seed)
    fg = ndimage.label(a, structure=np.ones((3, 3)))[1]
    lab, nb = ndimage.label(~np.pad(a, 1, constant_values=False))
    holes = nb - 1  # the padded border component is the outside
    assert geometry.euler_characteristic(a[None].astype(float), WALLS) == fg - holes


@pytest.mark.parametrize("seed", range(3))
def test_random_balls_3d_against_labelling(seed):
    rng = np.random.default_rng(100 + seed)
    n = 40
    phi = np.zeros((n, n, n))
    for _ in range(8):
        phi = np.maximum(phi, ball(n, rng.uniform(6, n - 6, 3), rng.uniform(2.5, 5.5)))
    count = ndimage.label(phi >= 0.5, structure=np.ones((3, 3, 3)))[1]
    assert geometry.euler_characteristic(phi, WALLS) == count


def test_mean_radius_of_tanh_droplets():
    """Eq. Rmoy_2D: I = 2 pi N <R> up to O(exp(-4R/W)) and lattice quadrature."""
    n, W = 200, 4.0
    y, x = np.mgrid[0:n, 0:n] + 0.5
    phi = np.zeros((n, n))
    radii = (20.0, 30.0, 25.0)
    centres = ((50.0, 50.0), (140.0, 60.0), (90.0, 150.0))
    for (cx, cy), R in zip(centres, radii):
        phi = np.maximum(phi, 0.5 * (1 + np.tanh(2 * (R - np.hypot(x - cx, y - cy)) / W)))
    phi = phi[None]
    N = geometry.euler_characteristic(phi, WALLS)
    assert N == 3
    assert abs(geometry.mean_radius(phi, W, N) - np.mean(radii)) < 0.01 * np.mean(radii)
    # 3D reading: I = 4 pi sum R^2
    n3 = 80
    z, y, x = np.mgrid[0:n3, 0:n3, 0:n3] + 0.5
    phi3 = 0.5 * (1 + np.tanh(2 * (15.0 - np.sqrt((x - 40) ** 2 + (y - 40) ** 2 + (z - 40) ** 2)) / W))
    assert geometry.euler_characteristic(phi3, WALLS) == 1
    assert abs(geometry.mean_radius(phi3, W, 1) - 15.0) < 0.02 * 15.0
