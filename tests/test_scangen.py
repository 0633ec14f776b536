"""The input generator: sizes, determinism, and the windowed ray casting
equal to testing every ray against every box."""
import numpy as np

from paper_2311_17604_amd import scangen


def test_window_casting_matches_all_rays():
    rng = np.random.Generator(np.random.PCG64(5))
    scene = scangen.wall_scene(rng, 40, 2.0, 30.0, 40.0, 20.0)
    R, C = 300, 500
    el, az = scangen._ray_dirs(R, C)
    for o in (np.array([0.0, 0.0, 1500.0]), np.array([3000.0, -2000.0, 1500.0])):
        ce, se = np.cos(el)[:, None], np.sin(el)[:, None]
        dx, dy = ce * np.cos(az)[None, :], ce * np.sin(az)[None, :]
        dz = np.broadcast_to(se, (R, C))
        t = scangen._exit(o, scene.close_lo, scene.close_hi, dx, dy, dz)
        tw = t.copy()
        for b in range(len(scene.box_lo)):
            t = np.minimum(t, scangen._slab(o, scene.box_lo[b], scene.box_hi[b], dx, dy, dz))
            i0, i1, jc = scangen._window(o, scene.box_lo[b], scene.box_hi[b], R, C)
            sub = np.ix_(np.arange(i0, i1), jc)
            tw[sub] = np.minimum(tw[sub], scangen._slab(o, scene.box_lo[b], scene.box_hi[b],
                                                        dx[sub], dy[sub], dz[sub]))
        assert np.isfinite(t).all()
        assert np.array_equal(t, tw)


def test_config1_shape_and_determinism():
    a = scangen.config(1)
    b = scangen.config(1)
    assert a.xyz.shape == (200_000, 3) and a.keep == 50_000 and a.k == 8
    assert np.array_equal(a.xyz, b.xyz)
    ext = a.xyz.max(0).astype(np.int64) - a.xyz.min(0)
    assert (ext < (1 << 21)).all()
    # the top row (400 rays straight up) is a near-duplicate cluster
    top = a.xyz[-400:]
    assert np.ptp(top[:, 0]) <= 2 and np.ptp(top[:, 1]) <= 2


def test_batch_scan_shapes():
    for s in range(10000, 10008):
        r, c, ratio = scangen.batch_scan_shape(s)
        assert 0.1 <= ratio <= 0.5
        assert 5_000 <= r * c <= 2_100_000


def test_merged_crop_equals_filtered_whole_cloud():
    """A crop of a merged cloud casts only the rays that can reach the box,
    and must give exactly the points of the whole cloud inside it, in the
    same order (the range noise is counter-based per ray)."""
    full = scangen.multi_station(4, 200, 300, 20, 200.0, 7)
    for lo, hi in (((-15000, -10000, -1000), (20000, 25000, 12000)),   # holds the first station
                   ((20000, -40000, -1000), (60000, 5000, 12000)),     # away from it
                   ((-3000, -3000, -1000), (3000, 3000, 12000))):
        m = ((full >= lo) & (full <= hi)).all(1)
        cr = scangen.multi_station(4, 200, 300, 20, 200.0, 7, crop=(lo, hi))
        assert m.sum() > 100
        assert np.array_equal(full[m], cr)


def test_ray_noise_counter_based():
    rays = np.arange(200_000)
    z = scangen.ray_noise(3, 2, rays, 2.0)
    assert abs(z.mean()) < 0.02 and abs(z.std() - 2.0) < 0.02
    sub = np.array([5, 77, 199_999, 1234])
    assert np.array_equal(scangen.ray_noise(3, 2, sub, 2.0), z[sub])
    assert not np.array_equal(scangen.ray_noise(3, 1, sub, 2.0), z[sub])
    assert not np.array_equal(scangen.ray_noise(4, 2, sub, 2.0), z[sub])


def test_merged_crop_workloads_small():
    for idx in (3, 5):
        w = scangen.config(idx, scale=0.0004, crop=True)
        assert w.name.endswith("/crop3m") and len(w.xyz) > 0
        assert ((w.xyz >= scangen.crop_box()[0]) & (w.xyz <= scangen.crop_box()[1])).all()
        assert w.keep == len(w.xyz) // (20 if idx == 3 else 50)
