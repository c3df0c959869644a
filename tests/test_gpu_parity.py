"""HIP path against the CPU oracle, element by element, on seeded inputs.

Integer stages must be bit-exact.  Colour deconvolution: the float c_H output
within 1e-5 relative of the FP64 oracle and Hq within 1 LSB (the device builds
its own log table, so a value sitting exactly on a rounding boundary may
round the other way).  Every stage after deconvolution is checked by
re-running the oracle from the GPU's own Hq.
"""
import numpy as np
import pytest

from paper_1405_7958_amd import synth
from tests.gpu_util import assert_equal, dev, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    from paper_1405_7958_amd import rtseg
    rtseg.lib()   # fails loudly if the HIP library is missing
    return rtseg


# ----------------------------------------------------------------------------
# colour deconvolution
# ----------------------------------------------------------------------------

def _check_deconv(rt, oracle, rgb, d):
    hq, ch = rt.rt_deconv(to_dev(rgb, d), want_ch=True)
    ohq, och = oracle.deconv(rgb, want_ch=True)
    ghq, gch = to_np(hq), to_np(ch)
    rel = np.abs(gch.astype(np.float64) - och) / np.maximum(np.abs(och), 1.0)
    assert rel.max() <= 1e-5, rel.max()
    diff = np.abs(ghq.astype(int) - ohq.astype(int))
    assert diff.max() <= 1
    return int((diff > 0).sum())


@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (17, 33), (512, 512), (301, 777)])
def test_deconv_random(rt, oracle, shape):
    d = dev()
    say("deconv", shape)
    rgb = synth.random_rgb(shape[0], shape[1], seed=shape[0] * 1000 + shape[1])
    assert _check_deconv(rt, oracle, rgb, d) <= max(2, rgb.size // 100000)


def test_deconv_exhaustive_all_rgb(rt, oracle):
    """All 2^24 RGB triples in one 4096 x 4096 image."""
    d = dev()
    say("deconv exhaustive")
    v = np.arange(1 << 24, dtype=np.uint32)
    rgb = np.stack([(v >> 16) & 255, (v >> 8) & 255, v & 255], -1).astype(np.uint8).reshape(4096, 4096, 3)
    n_lsb = _check_deconv(rt, oracle, rgb, d)
    assert n_lsb <= 64


def test_deconv_pitched(rt, oracle):
    import torch
    d = dev()
    say("deconv pitched")
    rgb = synth.random_rgb(40, 50, seed=3)
    big = torch.zeros((40, 64, 3), dtype=torch.uint8, device=d)
    big[:, :50] = to_dev(rgb, d)
    view = big[:, :50]
    hq = rt.rt_deconv(view)
    assert np.abs(to_np(hq).astype(int) - oracle.deconv(rgb).astype(int)).max() <= 1


def test_deconv_rejects_bad_args(rt):
    import torch
    d = dev()
    rgb = torch.zeros((4, 4, 3), dtype=torch.uint8, device=d)
    with pytest.raises(rt.RtError):
        rt.rt_deconv(rgb, stain=(1, 0, 0, 1, 0, 0, 0, 0, 0))   # H parallel to E: singular


# ----------------------------------------------------------------------------
# reconstruction
# ----------------------------------------------------------------------------

def _recon_case(seed, h, w, dtype, with_domain):
    r = np.random.Generator(np.random.PCG64(seed))
    if dtype == np.uint8:
        I = r.integers(0, 256, (h, w)).astype(np.uint8)
        J = np.where(r.random((h, w)) < 0.01, I, 0).astype(np.uint8)
    else:
        I = r.integers(-1000, 1000, (h, w)).astype(np.int32)
        J = np.where(r.random((h, w)) < 0.01, I, -2000).astype(np.int32)
    dom = (r.random((h, w)) < 0.9).astype(np.uint8) if with_domain else None
    return J, I, dom


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("dtype", [np.uint8, np.int32])
@pytest.mark.parametrize("shape", [(1, 1), (5, 7), (64, 64), (130, 67), (257, 300)])
def test_recon_random(rt, oracle, conn, dtype, shape):
    d = dev()
    for with_domain in (False, True):
        say("recon", conn, dtype.__name__, shape, with_domain)
        J, I, dom = _recon_case(shape[0] * 31 + shape[1] + conn, shape[0], shape[1], dtype, with_domain)
        got = rt.rt_morph_recon(to_dev(J, d), to_dev(I, d), to_dev(dom, d) if dom is not None else None, conn)
        exp = oracle.recon(J, I, dom, conn).astype(dtype)
        assert_equal(to_np(got), exp, f"recon conn={conn} {dtype.__name__} {shape} dom={with_domain}")


def test_recon_frame_marker_on_tile(rt, oracle):
    d = dev()
    say("recon frame marker 512")
    rgb, _, _ = synth.make_tile(synth.spec_small(0))
    hq = oracle.deconv(rgb)
    J = np.zeros_like(hq)
    J[0, :], J[-1, :], J[:, 0], J[:, -1] = hq[0, :], hq[-1, :], hq[:, 0], hq[:, -1]
    got = rt.rt_morph_recon(to_dev(J, d), to_dev(hq, d))
    assert_equal(to_np(got), oracle.recon(J, hq).astype(np.uint8), "frame recon")


def test_recon_spiral(rt, oracle):
    d = dev()
    say("recon spiral")
    s = (synth.spiral(150, 140) * 200).astype(np.uint8)
    J = np.zeros_like(s)
    J[0, 0] = 200
    for conn in (4, 8):
        got = rt.rt_morph_recon(to_dev(J, d), to_dev(s, d), None, conn)
        assert_equal(to_np(got), oracle.recon(J, s, None, conn).astype(np.uint8), f"spiral conn={conn}")


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("h,w,pad,offs", [(70, 129, 5, (1, 3, 2)), (130, 67, 0, (2, 0, 3)),
                                          (63, 63, 1, (3, 1, 1)), (125, 187, 3, (0, 2, 1))])
def test_recon_u8_strided_misaligned(rt, oracle, conn, h, w, pad, offs):
    """uint8 images at odd byte offsets with a pitch above the width, each
    image ending at the last byte of its buffer: the plain kernel stages rows
    through aligned dword loads clamped to the bytes of each row."""
    import torch
    d = dev()
    say("recon strided", conn, h, w, pad, offs)
    J, I, _ = _recon_case(h * 13 + w + pad, h, w, np.uint8, False)
    pitch = w + pad

    def view(img, off):
        buf = torch.zeros(off + (h - 1) * pitch + w, dtype=torch.uint8, device=d)
        v = torch.as_strided(buf, (h, w), (pitch, 1), off)
        v.copy_(torch.from_numpy(np.ascontiguousarray(img)).to(d))
        return v

    tJ, tI = view(J, offs[0]), view(I, offs[1])
    out = view(np.zeros_like(I), offs[2])
    # the binding needs marker, mask and output to share the pitch only
    rt.rt_morph_recon(tJ, tI, None, conn, out=out)
    assert_equal(to_np(out), oracle.recon(J, I, None, conn).astype(np.uint8), f"strided {h}x{w}+{pad} {offs}")


def test_recon_in_place(rt, oracle):
    d = dev()
    say("recon in place")
    J, I, _ = _recon_case(5, 90, 100, np.uint8, False)
    tJ = to_dev(J, d)
    rt.rt_morph_recon(tJ, to_dev(I, d), out=tJ)
    assert_equal(to_np(tJ), oracle.recon(J, I).astype(np.uint8), "in-place")


# ----------------------------------------------------------------------------
# FillHoles, BWLabel, AreaThreshold
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(1, 1), (1, 40), (40, 1), (33, 65), (129, 193), (200, 300), (1024, 1000)])
def test_fill_holes(rt, oracle, shape):
    d = dev()
    for p in (0.3, 0.55, 0.8):
        for bg in (4, 8):
            say("fill", shape, p, bg)
            b = synth.random_binary(shape[0], shape[1], p, seed=int(p * 100) + shape[1])
            got = rt.rt_fill_holes(to_dev(b, d), bg)
            assert_equal(to_np(got), oracle.fill_holes(b, bg), f"fill {shape} p={p} bg={bg}")
    rings = synth.nested_rings(97, 97)
    assert_equal(to_np(rt.rt_fill_holes(to_dev(rings, d))), oracle.fill_holes(rings), "rings")


@pytest.mark.parametrize("shape", [(1, 1), (1, 50), (50, 1), (31, 33), (64, 64), (129, 65), (65, 129), (300, 257),
                                   (1500, 1100)])
def test_ccl(rt, oracle, shape):
    d = dev()
    for p in (0.2, 0.45, 0.6, 0.9):
        for conn in (4, 8):
            say("ccl", shape, p, conn)
            b = synth.random_binary(shape[0], shape[1], p, seed=int(p * 100) + shape[0])
            lab, n = rt.rt_ccl(to_dev(b, d), conn)
            exp, nexp = oracle.ccl(b, conn)
            assert_equal(to_np(lab), exp, f"ccl {shape} p={p} conn={conn}")
            assert int(to_np(n)[0]) == nexp


def test_ccl_special(rt, oracle):
    d = dev()
    for name, b in [("checker", synth.checkerboard(100, 99)), ("spiral", synth.spiral(120, 130)),
                    ("rings", synth.nested_rings(80, 80)), ("zeros", np.zeros((70, 70), np.uint8)),
                    ("ones", np.ones((70, 70), np.uint8))]:
        for conn in (4, 8):
            say("ccl special", name, conn)
            lab, n = rt.rt_ccl(to_dev(b, d), conn)
            exp, nexp = oracle.ccl(b, conn)
            assert_equal(to_np(lab), exp, f"ccl {name} conn={conn}")
            assert int(to_np(n)[0]) == nexp


def test_area_filter(rt, oracle):
    d = dev()
    b = synth.random_binary(300, 280, 0.5, seed=77)
    lab, _ = oracle.ccl(b, 8)
    for lo, hi in [(1, 10 ** 8), (3, 30), (20, 1000), (7, 7)]:
        say("area", lo, hi)
        got, mask = rt.rt_area_filter(to_dev(lab, d), lo, hi)
        exp, emask, _ = oracle.area_filter(lab, lo, hi)
        assert_equal(to_np(got), exp, f"area {lo}-{hi}")
        assert_equal(to_np(mask), emask, f"area mask {lo}-{hi}")


# ----------------------------------------------------------------------------
# watershed
# ----------------------------------------------------------------------------

def _blobs(h, w, n, seed, rmin=3, rmax=12):
    r = np.random.Generator(np.random.PCG64(seed))
    yy, xx = np.mgrid[0:h, 0:w]
    fg = np.zeros((h, w), bool)
    for _ in range(n):
        cy, cx = r.uniform(0, h), r.uniform(0, w)
        a, b = r.uniform(rmin, rmax), r.uniform(rmin, rmax)
        t = r.uniform(0, np.pi)
        u = ((xx - cx) * np.cos(t) + (yy - cy) * np.sin(t)) / a
        v = (-(xx - cx) * np.sin(t) + (yy - cy) * np.cos(t)) / b
        fg |= u * u + v * v <= 1
    return fg.astype(np.uint8)


@pytest.mark.parametrize("case", [(64, 64, 6), (200, 180, 60), (333, 517, 300), (512, 512, 900)])
def test_watershed(rt, oracle, case):
    d = dev()
    h, w, n = case
    say("watershed", case)
    fg = _blobs(h, w, n, seed=h + w)
    lab, mask = rt.rt_watershed(to_dev(fg, d))
    elab, emask = oracle.watershed(fg)
    assert_equal(to_np(mask), emask, f"watershed mask {case}")
    assert_equal(to_np(lab), elab, f"watershed labels {case}")


def test_watershed_external_seeds(rt, oracle):
    d = dev()
    fg = _blobs(256, 256, 120, seed=9)
    r = np.random.Generator(np.random.PCG64(10))
    seeds = ((r.random(fg.shape) < 0.004) & (fg > 0)).astype(np.uint8)
    say("watershed seeds")
    lab, mask = rt.rt_watershed(to_dev(fg, d), to_dev(seeds, d))
    elab, emask = oracle.watershed(fg, seeds)
    assert_equal(to_np(lab), elab, "watershed external seeds")


def test_watershed_big_object(rt, oracle):
    """One component larger than the per-object LDS budget (global scratch path)."""
    d = dev()
    yy, xx = np.mgrid[0:200, 0:220]
    fg = (((yy - 100) ** 2 + (xx - 70) ** 2 <= 60 ** 2) | ((yy - 100) ** 2 + (xx - 150) ** 2 <= 55 ** 2)).astype(np.uint8)
    say("watershed big")
    lab, mask = rt.rt_watershed(to_dev(fg, d))
    elab, emask = oracle.watershed(fg)
    assert_equal(to_np(lab), elab, "watershed big object")


def test_watershed_every_object_class(rt, oracle):
    """Components of every size class in one image: small (crop <= 32^2),
    medium (<= 64^2), large LDS (<= 9312 px), global mid (<= 256^2) and the
    whole-tile global class; each made of two or three overlapping discs so
    the watershed has several seeds to split."""
    d = dev()
    yy, xx = np.mgrid[0:760, 0:900]

    def discs(*cs):
        m = np.zeros((760, 900), bool)
        for cy, cx, r in cs:
            m |= (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
        return m

    fg = (discs((20, 20, 9), (20, 36, 8)) |                      # small
          discs((60, 60, 18), (60, 95, 15)) |                    # medium
          discs((150, 60, 26), (150, 120, 24)) |                 # large (LDS)
          discs((330, 120, 70), (330, 250, 60), (380, 190, 40)) |  # global, mid slices
          discs((560, 560, 150), (560, 760, 120), (700, 650, 50)))  # global, whole-tile slices
    fg = fg.astype(np.uint8)
    say("watershed classes")
    lab, mask = rt.rt_watershed(to_dev(fg, d))
    elab, emask = oracle.watershed(fg)
    assert_equal(to_np(lab), elab, "watershed object classes")
    assert_equal(to_np(mask), emask, "watershed object classes mask")


def test_watershed_seed_counts(rt, oracle):
    """Grids of overlapping discs, one seed per disc, in crops of the small
    (<= 32^2) and the medium (<= 64^2) class: from 4 seeds to 25, so that
    both the register path (at most 8 seeds) and the plane path it defers
    to (more) run in both classes."""
    d = dev()
    H, W = 230, 260
    yy, xx = np.mgrid[0:H, 0:W]
    fg = np.zeros((H, W), bool)
    # (origin, rows, columns, radius, step): r 3 / step 6 grids stay in small crops, the others in medium ones
    grids = [((10, 10), 2, 2, 3, 6), ((10, 50), 2, 3, 3, 6), ((10, 100), 2, 4, 3, 6), ((10, 150), 3, 3, 3, 6),
             ((10, 200), 3, 4, 3, 6), ((80, 10), 2, 3, 6, 11), ((80, 70), 2, 4, 6, 11), ((80, 140), 3, 3, 5, 10),
             ((160, 10), 4, 4, 5, 10), ((160, 80), 5, 5, 5, 10)]
    for (y0, x0), ny, nx, r, step in grids:
        for i in range(ny):
            for j in range(nx):
                cy, cx = y0 + r + i * step, x0 + r + j * step
                fg |= (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
    fg = fg.astype(np.uint8)
    say("watershed seed counts")
    lab, mask = rt.rt_watershed(to_dev(fg, d))
    elab, emask = oracle.watershed(fg)
    assert_equal(to_np(lab), elab, "watershed seed counts")
    assert_equal(to_np(mask), emask, "watershed seed counts mask")
    # one piece per disc: 4 + 6 + 8 + 9 + 12 + 6 + 8 + 9 + 16 + 25
    assert len(np.unique(elab[elab > 0])) == 103


def test_watershed_all_foreground(rt, oracle):
    d = dev()
    fg = np.ones((40, 50), np.uint8)
    say("watershed all fg")
    lab, mask = rt.rt_watershed(to_dev(fg, d))
    elab, emask = oracle.watershed(fg)
    assert_equal(to_np(lab), elab, "watershed all foreground")


# ----------------------------------------------------------------------------
# whole tile
# ----------------------------------------------------------------------------

def _check_tile(rt, oracle, rgb, d, what):
    say("segment", what, rgb.shape)
    mask, lab, n, hq = rt.rt_segment_tile(to_dev(rgb, d), want_hq=True)
    ghq = to_np(hq)
    ohq = oracle.deconv(rgb)
    assert np.abs(ghq.astype(int) - ohq.astype(int)).max() <= 1
    emask, elab, en = oracle.segment_from_hq(ghq)
    assert_equal(to_np(mask), emask, f"{what} mask")
    assert_equal(to_np(lab), elab, f"{what} labels")
    assert int(to_np(n)[0]) == en
    return en


def test_segment_small_tile(rt, oracle):
    d = dev()
    rgb, gt, _ = synth.make_tile(synth.spec_small(0))
    assert _check_tile(rt, oracle, rgb, d, "small") > 50


@pytest.mark.parametrize("shape", [(1, 1), (1, 64), (37, 1), (100, 333), (129, 193), (700, 613)])
def test_segment_ragged(rt, oracle, shape):
    d = dev()
    spec = synth.TileSpec(w=shape[1], h=shape[0], seed=shape[0] + shape[1], n_nuclei=max(1, shape[0] * shape[1] // 2500),
                          amin=4, amax=14, cluster_frac=0.3, cluster_min=2, cluster_max=4, jitter=20)
    rgb, _, _ = synth.make_tile(spec)
    _check_tile(rt, oracle, rgb, d, f"ragged {shape}")


def test_segment_degenerate(rt, oracle):
    d = dev()
    white = np.full((96, 80, 3), 255, np.uint8)
    _check_tile(rt, oracle, white, d, "white")
    nuc = np.tile(np.array([120, 70, 150], np.uint8), (96, 80, 1))
    _check_tile(rt, oracle, nuc, d, "all nucleus colour")
    rnd = synth.random_rgb(200, 200, seed=4)
    _check_tile(rt, oracle, rnd, d, "random rgb")


def test_segment_dense_and_low_contrast(rt, oracle):
    d = dev()
    for i in range(40):
        spec = synth.spec_stream(i)
        if spec.w * spec.h > 1024 * 1024:
            continue
        rgb, _, _ = synth.make_tile(spec)
        _check_tile(rt, oracle, rgb, d, f"stream tile {i} {spec.kind}")


def test_segment_many_components_per_tile(rt, oracle):
    """About 320 components per 64 x 64 tile (kept 5 x 5 squares beside
    1-px dots that the first area filter erases): more than the per-tile
    statistics table holds, so part of the statistics and registrations take
    the direct path."""
    d = dev()
    rgb = np.empty((256, 256, 3), np.uint8)
    rgb[...] = (230, 180, 200)
    nuc = np.array([120, 70, 150], np.uint8)
    for cy in range(0, 256, 8):
        for cx in range(0, 256, 8):
            if ((cy // 8) + (cx // 8)) % 2 == 0:
                rgb[cy + 1:cy + 6, cx + 1:cx + 6] = nuc
            else:
                for dy in (1, 3, 5):
                    for dx in (1, 3, 5):
                        rgb[cy + dy, cx + dx] = nuc
    n = _check_tile(rt, oracle, rgb, d, "many components")
    assert n > 400


def test_segment_4k(rt, oracle):
    """The 4096 x 4096 workload, full-size, whole-image comparison."""
    d = dev()
    rgb, gt, _ = synth.make_tile(synth.spec_4k(0))
    n = _check_tile(rt, oracle, rgb, d, "4k")
    assert n > 5000


@pytest.mark.parametrize("knobs", [dict(recon_levels=3, recon_level_mode=0), dict(recon_levels=2, recon_level_mode=1),
                                   dict(recon_levels=8, recon_level_mode=1, recon_level_frac=300),
                                   dict(recon_levels=1, recon_level_mode=1, recon_level_frac=950),
                                   dict(recon_levels=5, recon_level_mode=1, recon_level_frac=1),
                                   dict(recon_levels=0), dict(objects_streams=0)])
def test_segment_level_choices(rt, oracle, knobs):
    """The threshold levels of the reconstruction's lower bound (and the
    per-object classes run one after the other instead of side by side)
    change only speed: every choice gives the oracle's result."""
    d = dev()
    ctx = rt.Context(0)
    for k, v in knobs.items():
        rt.rt_set_knob(k, v, ctx=ctx)
    for spec in (synth.spec_small(5), synth.spec_stream(2)):
        rgb, _, _ = synth.make_tile(spec)
        say("segment level choice", knobs, rgb.shape)
        mask, lab, n, hq = rt.rt_segment_tile(to_dev(rgb, d), want_hq=True, ctx=ctx)
        emask, elab, en = oracle.segment_from_hq(to_np(hq))
        assert_equal(to_np(mask), emask, f"{knobs} mask")
        assert_equal(to_np(lab), elab, f"{knobs} labels")
        assert int(to_np(n)[0]) == en


def test_segment_repeatable(rt):
    d = dev()
    rgb, _, _ = synth.make_tile(synth.spec_small(3))
    t = to_dev(rgb, d)
    say("repeat")
    m0, l0, n0 = rt.rt_segment_tile(t)
    for _ in range(3):
        m1, l1, n1 = rt.rt_segment_tile(t)
        assert_equal(to_np(l1), to_np(l0), "repeat labels")
