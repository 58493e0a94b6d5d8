"""Pins of the oracle's displacement tracking and MSD/VACF (Section 5.1):
ballistic particles crossing the periodic faces many times are unwrapped
exactly (the MSD is |v|^2 t^2 and the VACF |v|^2), and the tracker's result is
independent of how the trajectory is cut into snapshots."""
import math

import numpy as np


def test_ballistic_unwrapping(orc):
    rng = np.random.default_rng(4)
    N, L, dt = 500, 7.0, 0.05
    x0 = rng.random((3, N)) * L
    v = rng.normal(0, 3.0, (3, N))          # up to ~0.5 per step: well below L/2
    x_last = np.ascontiguousarray(x0.copy())
    disp = np.zeros((3, N))
    steps = 400                              # particles cross the box many times
    for n in range(1, steps + 1):
        x = np.mod(x0 + v * (n * dt), L)
        orc.track(x, L, x_last, disp)
    t = steps * dt
    assert np.allclose(disp, v * t, rtol=0, atol=1e-9)
    msd, vacf = orc.msd_vacf(disp, v, v)
    assert abs(msd - (v * v).sum() / N * t * t) <= 1e-9 * msd
    assert abs(vacf - (v * v).sum() / N) <= 1e-12 * vacf


def test_tracking_independent_of_snapshot_spacing(orc):
    rng = np.random.default_rng(5)
    N, L = 200, 5.0
    traj = [rng.random((3, N)) * L]
    for _ in range(60):
        traj.append(np.mod(traj[-1] + rng.normal(0, 0.3, (3, N)), L))
    out = []
    for stride in (1, 2):
        x_last = np.ascontiguousarray(traj[0].copy())
        disp = np.zeros((3, N))
        for x in traj[stride::stride]:
            orc.track(x, L, x_last, disp)
        out.append(disp)
    assert np.allclose(out[0], out[1], rtol=0, atol=1e-12)


def test_ballistic_unwrapping_cuboid(orc):
    """The same unwrapping with a different edge per axis: each component
    folds by its own edge (a shared edge would miscount the crossings)."""
    rng = np.random.default_rng(6)
    N, Lb, dt = 400, np.array([7.0, 4.5, 10.0]), 0.05
    x0 = rng.random((3, N)) * Lb[:, None]
    v = rng.normal(0, 3.0, (3, N))
    x_last = np.ascontiguousarray(x0.copy())
    disp = np.zeros((3, N))
    steps = 400
    for n in range(1, steps + 1):
        x = np.mod(x0 + v * (n * dt), Lb[:, None])
        orc.track(x, tuple(Lb), x_last, disp)
    assert np.allclose(disp, v * (steps * dt), rtol=0, atol=1e-9)
