"""GPU parity of the batched ragged-clip SOS path (one launch over every
clip, each with its own channel count, length and cascade) against the FP64
oracle, clip by clip; graph capture and the autotuner.

Tolerance: 1e-4 per-channel relative RMS (FP32 IIR)."""
import numpy as np
import pytest
import torch

import paper_2504_08624_amd as tfx
from paper_2504_08624_amd import design, lib, signals, workloads
from oracle import oracle as O
from tests.metrics import TOL_IIR_F32, assert_close

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _small_batch():
    """12 clips: lengths from 0 to ~3 tiles of the longest chunk, 1-5
    channels, 0-6 sections, one high-Q cascade."""
    g = signals.rng(501)
    Ns = [1, 7, 2048, 2049, 3071, 3072, 3073, 9000, 13000, 20000, 0, 4097]
    clips = []
    for i, N in enumerate(Ns):
        C = int(g.integers(1, 6))
        S = int(g.integers(0, 7)) if i != 5 else 3
        r_hi = 0.9995 if i == 5 else 0.99
        sec = design.random_sections(signals.rng(502, i), S, 0.5, r_hi).astype(np.float32).reshape(S, 5)
        x = signals.to_f32(np.stack([signals.white(N, (503, i, c)) for c in range(C)]).reshape(C, N))
        clips.append((x, sec))
    return clips


def _check(clips, ys, what):
    for i, ((x, sec), y) in enumerate(zip(clips, ys)):
        ref = O.sos(x, sec) if sec.shape[0] else x.astype(np.float64)
        if x.shape[1] == 0:
            assert tuple(y.shape) == x.shape
            continue
        assert_close(_cpu(y), ref, TOL_IIR_F32, "%s clip %d (C=%d N=%d S=%d)" % (what, i, *x.shape, sec.shape[0]))


@pytest.mark.parametrize("chunk", [16, 24, 32])
@pytest.mark.parametrize("order", [0, 1])
def test_batched_parity(chunk, order):
    clips = _small_batch()
    ys = tfx.sos_batched([_gpu(x) for x, _ in clips], [_gpu(s) for _, s in clips], {"chunk": chunk, "order": order})
    _check(clips, ys, "chunk=%d order=%d" % (chunk, order))


def test_batched_many_tiles_per_clip():
    # long clips: the look-back crosses 64-tile windows inside each clip
    clips = []
    for i, (C, N, S) in enumerate([(2, 300_000, 4), (1, 150_000, 6), (3, 70_000, 1)]):
        sec = design.random_sections(signals.rng(504, i), S, 0.5, 0.995).astype(np.float32)
        x = signals.to_f32(np.stack([signals.white(N, (505, i, c)) for c in range(C)]))
        clips.append((x, sec))
    for chunk in (16, 32):
        ys = tfx.sos_batched([_gpu(x) for x, _ in clips], [_gpu(s) for _, s in clips], {"chunk": chunk})
        _check(clips, ys, "long chunk=%d" % chunk)


def test_batched_graph_replay():
    clips = _small_batch()
    xs = [_gpu(x) for x, _ in clips]
    b = tfx.SosBatch(xs, [_gpu(s) for _, s in clips], {"chunk": 24, "order": 1})
    b.run()  # warm-up outside the capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            b.run()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        # new inputs each replay, written by ordinary eager work
        news = []
        for i, (x, sec) in enumerate(clips):
            xn = signals.to_f32(np.stack([signals.white(x.shape[1], (506, rep, i, c)) for c in range(x.shape[0])])
                                .reshape(x.shape))
            xs[i].copy_(_gpu(xn))
            news.append((xn, sec))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        _check(news, b.ys, "graph replay %d" % rep)


def test_batched_tune_picks_a_valid_config():
    clips = _small_batch()
    b = tfx.SosBatch([_gpu(x) for x, _ in clips], [_gpu(s) for _, s in clips])
    cfg, ms = b.tune(reps=2)
    assert cfg["chunk"] in (16, 24, 32) and cfg["order"] in (0, 1) and ms > 0
    ys = b.run()
    _check(clips, ys, "tuned %s" % cfg)


def test_batched_full_size_sampled_clips():
    # the ragged-batch workload at its full size (256 clips, 1-30 s @44.1 kHz,
    # 1-16 channels, 1-6 sections); the oracle checks 6 clips
    clips = workloads.ragged()
    ys = tfx.sos_batched([_gpu(x) for x, _ in clips], [_gpu(s) for _, s in clips], {"chunk": 24, "order": 1})
    rng = np.random.default_rng(507)
    for i in sorted(rng.choice(len(clips), 6, replace=False)):
        x, sec = clips[i]
        assert_close(_cpu(ys[i]), O.sos(x, sec), TOL_IIR_F32, "ragged clip %d (C=%d N=%d S=%d)"
                     % (i, x.shape[0], x.shape[1], sec.shape[0]))


def test_batched_argument_validation():
    x = _gpu(np.zeros((1, 10), np.float32))
    with pytest.raises(lib.TfxError, match="INVALID_ARG"):
        tfx.sos_batched([x], [_gpu(np.zeros((1, 5), np.float32))], {"chunk": 20})


@pytest.mark.parametrize("chunk", [16, 24])
def test_batched_long_cascades(chunk):
    """Clips with seven and eight sections (the longest cascade of the batch
    decides the form: at 24-sample chunks the matrix-core cascade) beside
    short ones, lengths across tile edges."""
    # peaking sections across the band: long cascades of unit-circle-zero
    # resonators have gains far below fp32 resolution (no fp32 method meets
    # 1e-4 there), peaking cascades stay well conditioned
    clips = []
    for i, (C, N, S) in enumerate([(3, 3 * 3072 + 5, 8), (1, 3072, 7), (2, 20_000, 2), (5, 777, 8), (2, 9000, 0)]):
        g = signals.rng(507, i)
        sec = (np.concatenate([design.peaking(f, q, gd, 44100.0) for f, q, gd in
                               zip(np.geomspace(200.0, 15000.0, S), g.uniform(0.7, 6.0, S), g.uniform(-9.0, 9.0, S))])
               if S else np.zeros((0, 5))).astype(np.float32).reshape(S, 5)
        x = signals.to_f32(np.stack([signals.white(N, (508, i, c)) for c in range(C)]).reshape(C, N))
        clips.append((x, sec))
    ys = tfx.sos_batched([_gpu(x) for x, _ in clips], [_gpu(s) for _, s in clips], {"chunk": chunk, "order": 1})
    _check(clips, ys, "long cascades chunk=%d" % chunk)


def test_batched_cascade_level_without_high_q():
    """Cascades of up to six sections and no high-Q section at 24-sample
    chunks (the cascade-level form: one look-back of the whole cascade
    state per tile); lengths across tile edges, odd channel counts."""
    clips = []
    for i, (C, N, S) in enumerate([(3, 3 * 3072 + 5, 6), (1, 3072, 1), (2, 20_000, 4), (5, 777, 3), (1, 9000, 0),
                                   (2, 40_000, 5)]):
        sec = design.random_sections(signals.rng(509, i), S, 0.5, 0.995).astype(np.float32).reshape(S, 5)
        x = signals.to_f32(np.stack([signals.white(N, (510, i, c)) for c in range(C)]).reshape(C, N))
        clips.append((x, sec))
    for order in (0, 1):
        ys = tfx.sos_batched([_gpu(x) for x, _ in clips], [_gpu(s) for _, s in clips], {"chunk": 24, "order": order})
        _check(clips, ys, "cascade-level order=%d" % order)
