"""GPU parity of the image block compression (section III-B, steps a-e)
against the FP64 oracle.

Steps (a)-(c) are FP32 arithmetic on uint8 pixels: every output within
2e-3 of the oracle (values up to 255; FP32 rounding is about 5e-5 here).
Steps (d) and (e) turn distances into integers (the nearest codeword, the
threshold tau): on images made of exact copies of k patterns every decision
has a wide margin and the codes and codebooks must agree exactly (codes) and
within 2e-3 (codewords); on smooth-noise photographs the codes must agree
wherever the oracle's decision margin is clear, and be valid (the GPU's pick
within the margin of the best) where it is not.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

ATOL = 2e-3


def _dp():
    import paper_1203_4938_amd as dp
    return dp


def _run(rgb, k, iters, tau):
    import torch
    dp = _dp()
    out = dp.img_compress(torch.from_numpy(rgb).cuda(), k, iters, tau)
    torch.cuda.synchronize()
    return {n: t.cpu().numpy() for n, t in out.items() if not n.startswith("_")}


def _front_ref(img):
    y, cb, cr = oracle.img_ycc(img)
    mean, act, dev = oracle.img_blocks(y)
    return y, cb, cr, mean, act, dev


def _check_front(g, b, img):
    y, cb, cr, mean, act, dev = _front_ref(img)
    errs = {"y": np.abs(g["y"][b] - y).max(), "cb": np.abs(g["cb"][b] - cb).max(),
            "cr": np.abs(g["cr"][b] - cr).max(), "mean": np.abs(g["mean"][b] - mean).max(),
            "act": np.abs(g["act"][b] - act).max(), "dev": np.abs(g["dev"][b] - dev).max()}
    assert max(errs.values()) <= ATOL, errs
    return errs, (y, cb, cr, mean, act, dev)


@pytest.mark.parametrize("shape", [(4, 4), (16, 64), (36, 100), (64, 132), (260, 516)])
def test_front_end_shapes(shape):
    """(a)-(c) on images whose sides are not multiples of the 64 x 16 tile,
    batch of 3."""
    h, w = shape
    rgb = synth.images_rgb(synth.BASE_SEED + 900, 3, h, w)
    g = _run(rgb, k=4, iters=1, tau=2.0)
    for b in range(3):
        errs, _ = _check_front(g, b, rgb[b])
    say(f"[img front] {h}x{w}: max errors " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))


def pattern_images(seed, B, h, w, k):
    """Grey images of 4x4 blocks that are exact copies of k random patterns,
    each block's pattern drawn uniformly except the blocks of raster rank
    floor(c nb / k), which take pattern c: with tau = 0 every block is a
    pattern block, so the k-means seeds are the k patterns, one each."""
    nb = (h // 4) * (w // 4)
    pick = synth.pattern_picks(seed + 1, B * nb, k).reshape(B, nb)
    for c in range(k):
        pick[:, (c * nb) // k] = c
    return synth.blocks_to_grey_rgb(synth.pattern_set(seed, k), pick.reshape(B, h // 4, w // 4))


@pytest.mark.parametrize("k,iters", [(8, 0), (8, 1), (16, 5), (64, 10), (256, 3), (5, 4), (17, 3),
                                     (100, 6)])
def test_pattern_images_exact(k, iters):
    """Images of exact copies of k random patterns, seeded one codeword per
    pattern: every block's nearest codeword is decided by a wide margin, so
    the GPU's codes equal the oracle's and its codebook the oracle's."""
    h, w, B = 64, 128, 2
    rgb = pattern_images(synth.BASE_SEED + 901 + k, B, h, w, k)
    g = _run(rgb, k=k, iters=iters, tau=0.0)
    for b in range(B):
        _, (y, cb, cr, mean, act, dev) = _check_front(g, b, rgb[b])
        book, P = oracle.img_kmeans(dev, act, 0.0, k, iters)
        code, margin = oracle.img_encode(dev, act, 0.0, book)
        assert P == dev.shape[0]
        assert margin.min() > 1.0, float(margin.min())
        assert np.array_equal(g["code"][b], code), int((g["code"][b] != code).sum())
        assert np.abs(g["codebook"][b] - book).max() <= ATOL
    say(f"[img patterns] k={k} iters={iters}: codes equal, codebook max err "
        f"{np.abs(g['codebook'][-1] - book).max():.1e}")


@pytest.mark.parametrize("k", [64, 150])
def test_pattern_images_exact_ragged_groups(k):
    """264 x 200 images: 3300 blocks, so the last workgroup of the assignment
    (1024 blocks, rounds of 256) ends inside its first round; k = 64 keeps
    the running cluster sums in LDS, k = 150 in the global partials."""
    h, w, B, iters = 264, 200, 2, 3
    rgb = pattern_images(synth.BASE_SEED + 941 + k, B, h, w, k)
    g = _run(rgb, k=k, iters=iters, tau=0.0)
    for b in range(B):
        _, (y, cb, cr, mean, act, dev) = _check_front(g, b, rgb[b])
        book, P = oracle.img_kmeans(dev, act, 0.0, k, iters)
        code, margin = oracle.img_encode(dev, act, 0.0, book)
        assert margin.min() > 1.0, float(margin.min())
        assert np.array_equal(g["code"][b], code), int((g["code"][b] != code).sum())
        assert np.abs(g["codebook"][b] - book).max() <= ATOL
    say(f"[img patterns] 264x200, k={k}: codes equal, codebook max err "
        f"{np.abs(g['codebook'][-1] - book).max():.1e}")


@pytest.mark.parametrize("k", [64, 200])
def test_photo_pipeline_is_deterministic(k):
    """Photographs (near ties, sums whose rounding depends on their order):
    two runs give the same bits in every output, with the cluster sums in LDS
    (k = 64) and in the global partials (k = 200)."""
    h, w, B, iters, tau = 512, 512, 2, 6, 8.0
    rgb = synth.images_rgb(synth.BASE_SEED + 951, B, h, w)
    g1 = _run(rgb, k=k, iters=iters, tau=tau)
    g2 = _run(rgb, k=k, iters=iters, tau=tau)
    for n in g1:
        assert np.array_equal(g1[n], g2[n]), n
    say(f"[img determinism] k={k}: two runs bitwise equal")


def test_graph_replays_match_direct_launches():
    """IMG_F_GRAPH: the launch sequence replayed from a HIP graph on the same
    buffers, three times with eager work between the replays and the outputs
    overwritten before each, gives exactly the outputs of the direct launches
    (pattern images: every cluster sum adds copies of one vector, so no
    rounding depends on the order of the additions)."""
    import ctypes

    import torch
    dp = _dp()
    k, iters, B, h, w = 16, 4, 2, 64, 128
    rgb = torch.from_numpy(pattern_images(synth.BASE_SEED + 930, B, h, w, k)).cuda()
    ref = dp.img_compress(rgb, k, iters, 0.0)
    torch.cuda.synchronize()
    ref_np = {n: t.cpu().numpy() for n, t in ref.items() if not n.startswith("_")}
    out = {n: torch.empty_like(t) for n, t in ref.items() if not n.startswith("_")}
    ws = torch.empty_like(ref["_workspace"])
    names = ("y", "cb", "cr", "mean", "act", "dev", "codebook", "code")
    o = dp.ImgOut(*(out[n].data_ptr() for n in names))
    d = dp.ImgDesc(height=h, width=w, batch=B, k=k, iters=iters, tau=0.0, flags=dp.IMG_F_GRAPH)
    for rep in range(3):
        for t in out.values():
            t.fill_(7)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        st = dp._lib.img_compress(ctypes.byref(d), ctypes.c_void_p(rgb.data_ptr()), ctypes.byref(o),
                                  ctypes.c_void_p(ws.data_ptr()), None)
        assert st == dp.FFT_OK, dp.fft_last_error()
        torch.cuda.synchronize()
        for n in names:
            assert np.array_equal(out[n].cpu().numpy(), ref_np[n]), (rep, n)
        say(f"[img graph] replay {rep}: outputs equal the direct launches (junk {float(junk):.1f})")


def test_graph_cache_beyond_its_capacity():
    """IMG_F_GRAPH on 10 output buffer sets (more than the 8 graphs kept),
    then the first set again (rebuilt after its eviction): every call equals
    the direct launches exactly (pattern images)."""
    import ctypes

    import torch
    dp = _dp()
    k, iters, B, h, w = 8, 2, 1, 32, 64
    rgb = torch.from_numpy(pattern_images(synth.BASE_SEED + 931, B, h, w, k)).cuda()
    ref = dp.img_compress(rgb, k, iters, 0.0)
    torch.cuda.synchronize()
    names = ("y", "cb", "cr", "mean", "act", "dev", "codebook", "code")
    ref_np = {n: ref[n].cpu().numpy() for n in names}
    sets = []
    for _ in range(10):
        out = {n: torch.empty_like(ref[n]) for n in names}
        sets.append((out, dp.ImgOut(*(out[n].data_ptr() for n in names)),
                     torch.empty_like(ref["_workspace"])))
    d = dp.ImgDesc(height=h, width=w, batch=B, k=k, iters=iters, tau=0.0, flags=dp.IMG_F_GRAPH)
    for i in list(range(10)) + [0]:
        out, o, ws = sets[i]
        for t in out.values():
            t.fill_(5)
        st = dp._lib.img_compress(ctypes.byref(d), ctypes.c_void_p(rgb.data_ptr()), ctypes.byref(o),
                                  ctypes.c_void_p(ws.data_ptr()), None)
        assert st == dp.FFT_OK, dp.fft_last_error()
        torch.cuda.synchronize()
        for n in names:
            assert np.array_equal(out[n].cpu().numpy(), ref_np[n]), (i, n)


def _valid_codes(gcode, dev, act, tau, book, act_eps=1e-3, rel_eps=1e-4):
    """Codes the oracle would accept: equal to its own, or a decision within
    FP32's reach of a tie (activity within act_eps of tau, or a codeword whose
    distance is within rel_eps of the best)."""
    code, margin = oracle.img_encode(dev, act, tau, book)
    bad = np.nonzero(gcode != code)[0]
    for i in bad:
        if abs(act[i] - tau) <= act_eps:
            continue
        if gcode[i] >= 1 and code[i] >= 1:
            d = ((dev[i][None, :] - book) ** 2).sum(-1)
            best = d.min()
            if d[gcode[i] - 1] <= best + rel_eps * (1.0 + best):
                continue
        return False, int(i)
    return True, len(bad)


def test_photo_encode_with_oracle_codebook():
    """(e) alone on smooth-noise colour photographs, with the oracle's
    codebook: every code matches unless the decision is a near tie."""
    import torch
    dp = _dp()
    h, w, B, k, tau = 256, 384, 2, 32, 8.0
    rgb = synth.images_rgb(synth.BASE_SEED + 910, B, h, w)
    g = _run(rgb, k=k, iters=0, tau=tau)
    books, refs = [], []
    for b in range(B):
        _, ref = _check_front(g, b, rgb[b])
        book, _ = oracle.img_kmeans(ref[5], ref[4], tau, k, 6)
        books.append(book.astype(np.float32))
        refs.append(ref)
    code = dp.img_encode(torch.from_numpy(g["dev"]).cuda(),
                         torch.from_numpy(np.ascontiguousarray(g["act"].reshape(B, -1))).cuda(),
                         torch.from_numpy(np.stack(books)).cuda(), h, w, tau).cpu().numpy()
    for b in range(B):
        ok, n = _valid_codes(code[b], refs[b][5], refs[b][4].reshape(-1), tau,
                             books[b].astype(np.float64))
        assert ok, f"image {b}: block {n} has an invalid code"
        say(f"[img encode] image {b}: {n} near-tie codes differ, all valid")


def test_photo_pipeline_seeds_and_lloyd():
    """The whole pipeline on photographs: with tau in a gap of the activities
    (no block within 1e-3 of it) the seeds (0 iterations) equal the oracle's;
    after Lloyd iterations the GPU's codes are the nearest codewords of its
    own codebook, and its objective is no larger than at the seeds."""
    h, w, B, k = 256, 256, 2, 64
    rgb = synth.images_rgb(synth.BASE_SEED + 920, B, h, w)
    g0 = _run(rgb, k=k, iters=0, tau=0.0)
    acts = np.sort(g0["act"].reshape(-1))
    gaps = np.diff(acts)
    mid = np.argmax(gaps[len(gaps) // 3: 2 * len(gaps) // 3]) + len(gaps) // 3
    tau = float(0.5 * (acts[mid] + acts[mid + 1]))
    assert gaps[mid] > 2e-3, gaps[mid]
    g0 = _run(rgb, k=k, iters=0, tau=tau)
    g = _run(rgb, k=k, iters=8, tau=tau)
    for b in range(B):
        _, (y, cb, cr, mean, act, dev) = _check_front(g, b, rgb[b])
        seeds, P = oracle.img_kmeans(dev, act, tau, k, 0)
        assert np.abs(g0["codebook"][b] - seeds).max() <= ATOL
        gdev = g["dev"][b].astype(np.float64)
        gbook = g["codebook"][b].astype(np.float64)
        ok, n = _valid_codes(g["code"][b], gdev, g["act"][b].reshape(-1).astype(np.float64), tau,
                             gbook)
        assert ok, f"image {b}: block {n}"
        pat = act.reshape(-1) >= tau
        sse = lambda bk: ((gdev[pat][:, None, :] - bk[None]) ** 2).sum(-1).min(axis=1).sum()
        assert sse(gbook) <= sse(g0["codebook"][b].astype(np.float64)) * (1 + 1e-5)
        say(f"[img pipeline] image {b}: {P} pattern blocks, tau {tau:.3f}, objective "
            f"{sse(g0['codebook'][b].astype(np.float64)):.4g} -> {sse(gbook):.4g}")


@pytest.mark.parametrize("k,h,w", [(1, 64, 64), (2, 4, 8), (3, 4, 4)])
def test_small_k_and_tiny_images(k, h, w):
    """Edge cases of the assignment: one codeword (every pattern block in
    cluster 0), images of one or two 4x4 blocks (one partial round of the
    first workgroup, most lanes past the last block); tau = 0, so every block
    with any gradient is a pattern block."""
    B, iters = 3, 2
    rgb = synth.images_rgb(synth.BASE_SEED + 961 + k, B, h, w)
    g = _run(rgb, k=k, iters=iters, tau=0.0)
    for b in range(B):
        _, (y, cb, cr, mean, act, dev) = _check_front(g, b, rgb[b])
        book, P = oracle.img_kmeans(dev, act, 0.0, k, iters)
        assert np.abs(g["codebook"][b] - book).max() <= ATOL, b
        ok, n = _valid_codes(g["code"][b], g["dev"][b].astype(np.float64),
                             g["act"][b].reshape(-1).astype(np.float64), 0.0,
                             g["codebook"][b].astype(np.float64))
        assert ok, (b, n)
    say(f"[img small] k={k} {h}x{w}: codebooks within {ATOL}, codes valid")


def test_batch_zero_and_uniform_image():
    """An empty batch is a no-op; a flat image has no pattern block (all codes
    0, zero codebook)."""
    import torch
    dp = _dp()
    d = dp.ImgDesc(height=16, width=16, batch=0, k=4, iters=2, tau=1.0)
    o = dp.ImgOut()
    assert dp._lib.img_compress(d, None, o, None, None) == dp.FFT_OK
    rgb = np.full((1, 32, 64, 3), 90, np.uint8)
    g = _run(rgb, k=4, iters=3, tau=0.5)
    assert np.all(g["code"] == 0) and np.all(g["codebook"] == 0)
    assert np.allclose(g["y"], 90.0, atol=1e-4) and np.allclose(g["cb"], 128.0, atol=1e-4)


def test_bench_batch_every_image():
    """The benchmark's workload: 16 colour photographs of 2048 x 2048, k = 64,
    8 iterations, tau = 8 (about two blocks in five keep their mean only):
    steps (a)-(c) of every image against the oracle, and every code a valid
    nearest codeword of the GPU's codebook."""
    h = w = 2048
    B, k, iters, tau = 16, 64, 8, 8.0
    rgb = synth.images_rgb(synth.BASE_SEED + 7, B, h, w)
    g = _run(rgb, k=k, iters=iters, tau=tau)
    worst = 0.0
    for b in range(B):
        errs, _ = _check_front(g, b, rgb[b])
        worst = max(worst, max(errs.values()))
        ok, n = _valid_codes(g["code"][b], g["dev"][b].astype(np.float64),
                             g["act"][b].reshape(-1).astype(np.float64), tau,
                             g["codebook"][b].astype(np.float64))
        assert ok, f"image {b}: block {n}"
    say(f"[img bench] 16 x 2048^2: front-end max error {worst:.1e}, codes valid")
