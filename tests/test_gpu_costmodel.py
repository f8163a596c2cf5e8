"""GPU parity of the cost-model MLP kernels against the fp64 oracle.

Each GEMM is checked on its own: the oracle takes the GPU's own inputs to
that GEMM, rounds them to bf16 exactly as the kernel does, and computes the
products in fp64.  The remaining difference is the kernel's fp32
accumulation, bounded by K * 2^-23 * sum_k |a_k b_k| (plus one fp32
rounding of the bias add), which is the tolerance used.
"""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_04349_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(hb):
    c = hb.hb_create(0, allocator="torch")
    yield c
    c.close()


def flat(p):
    return np.concatenate([p[k].ravel() for k, _ in mlp.SHAPES]).astype(np.float32)


def unflat(v):
    p, o = {}, 0
    for k, s in mlp.SHAPES:
        n = int(np.prod(s))
        p[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(s)
        o += n
    return p


def check_gemm(a, b, got, bias=None, mask=None):
    """got ~ bf16(a) @ bf16(b) (+ bias) (masked), within the fp32 bound."""
    ab, bb = mlp.bf16_round(a), mlp.bf16_round(b)
    want = ab @ bb
    bound = np.abs(ab) @ np.abs(bb) * (a.shape[1] * 2.0 ** -23)
    if bias is not None:
        want = want + bias
        bound = bound + np.abs(want) * 2.0 ** -23
    if mask is not None:
        want = np.where(mask > 0, want, 0.0)
        bound = np.where(mask > 0, bound, 0.0)
    err = np.abs(got.astype(np.float64) - want)
    assert np.all(err <= bound + 1e-30), float((err - bound).max())


def test_forward_backward_per_gemm(hb, ctx):
    print("[gpu-case] costmodel trace", flush=True)
    r = np.random.default_rng(3)
    n = 40
    x = r.normal(size=(n, 16)).astype(np.float32)
    t = r.normal(size=(n, 2)).astype(np.float32)
    p64 = mlp.init_params(9)
    for k in ("b1", "b2", "b3"):
        p64[k] = r.normal(size=p64[k].shape) * 0.1
    w = flat(p64)
    hb.hb_costmodel_set_params(ctx, w)
    assert np.array_equal(hb.hb_costmodel_get_params(ctx), w)
    p = unflat(w)
    tr = hb.hb_costmodel_trace(ctx, x, t)
    x64 = x.astype(np.float64)
    check_gemm(x64, p["W1"], tr["z1"], bias=p["b1"])
    assert np.array_equal(tr["h1"], np.maximum(tr["z1"], 0))
    check_gemm(tr["h1"].astype(np.float64), p["W2"], tr["z2"], bias=p["b2"])
    assert np.array_equal(tr["h2"], np.maximum(tr["z2"], 0))
    check_gemm(tr["h2"].astype(np.float64), p["W3"], tr["y"], bias=p["b3"])
    dy = 2.0 * (tr["y"].astype(np.float64) - t) / (n * 2)
    assert np.allclose(tr["dy"], dy, rtol=1e-6, atol=1e-12)
    g = unflat(tr["grad"])
    check_gemm(tr["h2"].T.astype(np.float64), tr["dy"].astype(np.float64), g["W3"])
    assert np.allclose(g["b3"], tr["dy"].astype(np.float64).sum(0), rtol=1e-5, atol=1e-9)
    check_gemm(tr["dy"].astype(np.float64), p["W3"].T, tr["dz2"], mask=tr["z2"])
    check_gemm(tr["h1"].T.astype(np.float64), tr["dz2"].astype(np.float64), g["W2"])
    check_gemm(tr["dz2"].astype(np.float64), p["W2"].T, tr["dz1"], mask=tr["z1"])
    check_gemm(x64.T, tr["dz1"].astype(np.float64), g["W1"])
    assert np.allclose(g["b1"], tr["dz1"].astype(np.float64).sum(0), rtol=1e-5, atol=1e-9)


def test_gradients_close_to_fp64_backprop(hb, ctx):
    # end to end: the bf16 forward/backward is a close approximation of the
    # fp64 gradients of the same weights (direction and magnitude)
    r = np.random.default_rng(4)
    x = r.normal(size=(64, 16)).astype(np.float32)
    t = r.normal(size=(64, 2)).astype(np.float32)
    p64 = mlp.init_params(5)
    w = flat(p64)
    hb.hb_costmodel_set_params(ctx, w)
    tr = hb.hb_costmodel_trace(ctx, x, t)
    p = unflat(w)
    y, cache = mlp.forward(p, x.astype(np.float64))
    gw = flat(mlp.backward(p, y, t.astype(np.float64), cache)).astype(np.float64)
    gg = tr["grad"].astype(np.float64)
    cos = gg @ gw / np.linalg.norm(gg) / np.linalg.norm(gw)
    assert cos > 0.999
    assert abs(np.linalg.norm(gg) / np.linalg.norm(gw) - 1) < 0.02


def test_adam_step_matches_oracle(hb, ctx):
    r = np.random.default_rng(6)
    w = flat(mlp.init_params(2))
    hb.hb_costmodel_set_params(ctx, w)
    p = unflat(w)
    st = {}
    for step in range(3):
        g = r.normal(size=w.size).astype(np.float32) * 10.0 ** r.integers(-3, 2)
        hb.hb_costmodel_adam_step(ctx, g, 1e-3)
        mlp.adam_step(p, unflat(g), st, lr=1e-3)
        got = hb.hb_costmodel_get_params(ctx).astype(np.float64)
        assert np.allclose(got, flat(p).astype(np.float64), rtol=1e-5, atol=1e-7), step


def test_training_fits_a_smooth_target(hb, ctx):
    print("[gpu-case] costmodel train", flush=True)
    r = np.random.default_rng(8)
    x = r.uniform(-1, 1, size=(8192, 16)).astype(np.float32)
    wt = r.normal(size=(16, 2))
    t = (np.tanh(x @ wt) * 0.5).astype(np.float32)
    hb.hb_costmodel_init(ctx, 11)
    y0 = hb.hb_costmodel_predict(ctx, x)
    l0 = float(np.mean((y0 - t) ** 2))
    loss = hb.hb_costmodel_train(ctx, x, t, epochs=30, batch=512, lr=2e-3)
    y1 = hb.hb_costmodel_predict(ctx, x)
    l1 = float(np.mean((y1 - t) ** 2))
    assert l1 < 0.1 * l0, (l0, l1)
    assert abs(loss - l1) < 0.5 * l1 + 1e-3


def test_fused_inference_matches_layerwise_forward(hb, ctx):
    """hb_costmodel_predict runs one fused kernel (activations in
    registers); the trace runs the layer-by-layer GEMMs checked above.
    Both round every operand to bf16 and accumulate in fp32, so they agree
    except where a one-ulp accumulation difference flips an activation's
    bf16 rounding."""
    print("[gpu-case] fused inference", flush=True)
    r = np.random.default_rng(21)
    x = r.normal(size=(3000, 16)).astype(np.float32)   # not a multiple of 16 rows
    t = np.zeros((3000, 2), dtype=np.float32)
    hb.hb_costmodel_init(ctx, 5)
    fused = hb.hb_costmodel_predict(ctx, x).astype(np.float64)
    tr = hb.hb_costmodel_trace(ctx, x, t)
    lay = tr["y"].astype(np.float64)
    d = np.abs(fused - lay)
    scale = np.abs(lay).max() + 1e-3
    assert np.median(d) <= 1e-6 * scale, float(np.median(d))
    assert d.max() <= 2e-2 * scale, float(d.max())
    # and against the fp64 oracle forward with bf16 operands, loosely
    p = unflat(hb.hb_costmodel_get_params(ctx))
    y64, _ = mlp.forward(p, x.astype(np.float64))
    assert np.abs(fused - y64).max() <= 0.05 * (np.abs(y64).max() + 1e-3)


def test_save_load_round_trip(hb, ctx, tmp_path):
    """hb_costmodel_save / hb_costmodel_load through the C ABI: the loaded
    parameters are bit-identical in a fresh context and predict the same;
    a corrupted, truncated or foreign file is refused and leaves the
    context's model as it was."""
    print("[gpu-case] costmodel save/load", flush=True)
    r = np.random.default_rng(31)
    x = r.normal(size=(700, 16)).astype(np.float32)
    t = (np.tanh(x[:, :2]) * 0.5).astype(np.float32)
    hb.hb_costmodel_init(ctx, 17)
    hb.hb_costmodel_train(ctx, x, t, epochs=3, batch=128, lr=1e-3)
    want = hb.hb_costmodel_get_params(ctx)
    path = str(tmp_path / "model.hbcm")
    hb.hb_costmodel_save(ctx, path)
    raw = open(path, "rb").read()
    assert raw[:8] == b"HBCMODEL" and len(raw) == 8 + 6 * 4 + hb.HB_MLP_PARAMS * 4 + 8
    assert np.array_equal(np.frombuffer(raw[32:32 + hb.HB_MLP_PARAMS * 4], dtype="<f4"), want)

    other = hb.hb_create(0, allocator="torch")
    try:
        with pytest.raises(hb.HbError) as e:   # nothing to save yet
            hb.hb_costmodel_save(other, str(tmp_path / "none.hbcm"))
        assert e.value.status == hb.HB_ERR_STATE
        hb.hb_costmodel_load(other, path)
        got = hb.hb_costmodel_get_params(other)
        assert got.view(np.uint32).tolist() == want.view(np.uint32).tolist()
        assert np.array_equal(hb.hb_costmodel_predict(other, x), hb.hb_costmodel_predict(ctx, x))
        # refused files leave the loaded model untouched
        bad = bytearray(raw)
        bad[40] ^= 1   # one parameter bit: checksum mismatch
        cases = {"flip.hbcm": bytes(bad), "short.hbcm": raw[:-9], "long.hbcm": raw + b"\0",
                 "magic.hbcm": b"HBXMODEL" + raw[8:]}
        shape = bytearray(raw)
        shape[16] = 32   # hidden width 32
        cases["shape.hbcm"] = bytes(shape)
        for name, data in cases.items():
            p = tmp_path / name
            p.write_bytes(data)
            with pytest.raises(hb.HbError) as e:
                hb.hb_costmodel_load(other, str(p))
            assert e.value.status == hb.HB_ERR_INVALID_ARG, name
        with pytest.raises(hb.HbError):
            hb.hb_costmodel_load(other, str(tmp_path / "missing.hbcm"))
        assert np.array_equal(hb.hb_costmodel_get_params(other), want)
    finally:
        other.close()
