"""Antenna layouts and earth-rotation synthesis of uvw tracks (inputs only).

Earth-rotation synthesis follows the textbook relations (Thompson, Moran & Swenson,
"Interferometry and Synthesis in Radio Astronomy", eqs. 4.1 and 4.15): local
east/north/up antenna offsets are rotated to equatorial XYZ at latitude phi, and
for hour angle H and declination delta each baseline (X, Y, Z) projects to

    u =  sin H X + cos H Y
    v = -sin d cos H X + sin d sin H Y + cos d Z
    w =  cos d cos H X - cos d sin H Y + sin d Z

in metres.  One row per baseline p < q per integration, time-major ordering
(row = t * n_baselines + b).
"""

import numpy as np

C_LIGHT = 299_792_458.0  # m/s


def n_baselines(n_ant):
    return n_ant * (n_ant - 1) // 2


def layout_uniform_disc(rng, n_ant, radius_m):
    """n_ant antennas uniform in a disc of the given radius (east, north, up)."""
    r = radius_m * np.sqrt(rng.random(n_ant))
    th = 2.0 * np.pi * rng.random(n_ant)
    return np.stack([r * np.cos(th), r * np.sin(th), np.zeros(n_ant)], axis=1)


def layout_vla_y(rng, n_per_arm=9, arm_len_m=21_000.0, r_min_m=40.0, jitter=0.02):
    """VLA-like Y: three arms 120 degrees apart, antennas log-spaced to arm_len."""
    d = np.geomspace(r_min_m, arm_len_m, n_per_arm)
    pos = []
    for k, az in enumerate(np.deg2rad([5.0, 125.0, 245.0])):
        dd = d * (1.0 + jitter * rng.standard_normal(n_per_arm))
        pos.append(np.stack([dd * np.sin(az), dd * np.cos(az), np.zeros(n_per_arm)], axis=1))
    return np.concatenate(pos, axis=0)


def layout_meerkat_like(rng, n_core=48, core_radius_m=500.0, n_spiral=16,
                        r_in_m=1_000.0, r_out_m=8_000.0, n_arms=3, twist=1.5):
    """Dense uniform core plus antennas on three logarithmic spirals."""
    core = layout_uniform_disc(rng, n_core, core_radius_m)
    per_arm = [n_spiral // n_arms + (1 if a < n_spiral % n_arms else 0) for a in range(n_arms)]
    pts = []
    for a, n in enumerate(per_arm):
        r = np.geomspace(r_in_m, r_out_m, n) * (1.0 + 0.03 * rng.standard_normal(n))
        th = 2.0 * np.pi * a / n_arms + twist * np.log(r / r_in_m)
        pts.append(np.stack([r * np.cos(th), r * np.sin(th), np.zeros(n)], axis=1))
    return np.concatenate([core] + pts, axis=0)


def enu_to_xyz(enu, lat_rad):
    e, n, u = enu[:, 0], enu[:, 1], enu[:, 2]
    x = -np.sin(lat_rad) * n + np.cos(lat_rad) * u
    y = e
    z = np.cos(lat_rad) * n + np.sin(lat_rad) * u
    return np.stack([x, y, z], axis=1)


def earth_rotation_uvw(enu, lat_rad, dec_rad, hour_angles_rad):
    """uvw [n_int * n_bl, 3] in metres, time-major."""
    xyz = enu_to_xyz(enu, lat_rad)
    p, q = np.triu_indices(len(enu), k=1)
    b = xyz[q] - xyz[p]  # [n_bl, 3]
    H = np.asarray(hour_angles_rad)[:, None]
    X, Y, Z = b[None, :, 0], b[None, :, 1], b[None, :, 2]
    sd, cd = np.sin(dec_rad), np.cos(dec_rad)
    u = np.sin(H) * X + np.cos(H) * Y
    v = -sd * np.cos(H) * X + sd * np.sin(H) * Y + cd * Z
    w = cd * np.cos(H) * X - cd * np.sin(H) * Y + sd * Z
    return np.stack([u, v, w], axis=-1).reshape(-1, 3)
