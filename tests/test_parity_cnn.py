"""The tile CNN's GPU forward / backward (BF16 matrix cores, FP32 sums)
against the float64 oracle that rounds to BF16 at the same points; the
training step; tile normalisation; proposals."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_09784_amd import fh
    fh.lib()
    return torch.device("cuda:0")


def _tiles(rng, B):
    # normalised-count-like inputs: mostly N(0,1), a few bright lines
    t = rng.normal(size=(B, 64, 64))
    for b in range(0, B, 2):
        r = rng.integers(0, 64)
        t[b, r, :] += 4.0
    return t


def _to_bf16(dev, t):
    import torch
    return torch.from_numpy(np.asarray(t, dtype=np.float32)).to(dev).to(torch.bfloat16).contiguous()


def _layer_slices():
    sizes = [16 * 9, 16, 32 * 9 * 16, 32, 64 * 9 * 32, 64, 64 * 9 * 64, 64, 64, 1]
    names = ["w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4", "w5", "b5"]
    out, o = {}, 0
    for n, s in zip(names, sizes):
        out[n] = slice(o, o + s)
        o += s
    return out


@pytest.mark.parametrize("seed,B", [(0, 2), (1, 5), (2, 8)])
def test_forward_backward_match_oracle(dev, seed, B):
    import torch
    from paper_1810_09784_amd import fh
    from oracle import cnn as N
    rng = np.random.default_rng(seed)
    th = N.init_params(rng).astype(np.float32).astype(np.float64)
    tiles = _tiles(rng, B)
    labels = (np.arange(B) % 2 == 0).astype(np.float64)
    net = fh.CNN(max_batch=8)
    net.set_params(th)
    xt = _to_bf16(dev, tiles)
    logits = net.forward(xt).cpu().numpy().astype(np.float64)
    loss = net.backward(torch.from_numpy(labels.astype(np.float32)).to(dev)).cpu().numpy()[0]
    torch.cuda.synchronize()
    _, g = net.get_params()
    # the oracle sees exactly the BF16 tiles the GPU saw
    ref_loss, ref_g, ref_logit = N.loss_and_grad(th, xt.float().cpu().numpy(), labels, bf=True)
    assert np.max(np.abs(logits - ref_logit)) <= 2e-3 * (1.0 + np.max(np.abs(ref_logit))), (logits, ref_logit)
    assert abs(loss - ref_loss) <= 2e-3 * (1 + abs(ref_loss))
    for name, sl in _layer_slices().items():
        rg = ref_g[sl]
        err = np.linalg.norm(g[sl] - rg) / max(np.linalg.norm(rg), 1e-12)
        assert err <= 1e-2, (name, err)


def test_training_reduces_loss(dev):
    # bright-line tiles against noise tiles: a few Adam steps must separate them
    import torch
    from paper_1810_09784_amd import fh
    from oracle import cnn as N
    rng = np.random.default_rng(5)
    net = fh.CNN(max_batch=32)
    net.set_params(N.init_params(rng))
    losses = []
    for it in range(80):
        t = rng.normal(size=(32, 64, 64))
        y = (np.arange(32) % 2).astype(np.float32)
        for b in range(32):
            if y[b] > 0:
                r = rng.integers(0, 64)
                t[b, r, :] += 1.5
        net.forward(_to_bf16(dev, t))
        losses.append(float(net.backward(torch.from_numpy(y).to(dev)).item()))
        net.step(3e-4)
    assert np.mean(losses[-10:]) < 0.85 * np.mean(losses[:5]), losses


def test_tiles_are_row_normalised(dev):
    import torch
    from paper_1810_09784_amd import fh
    rng = np.random.default_rng(6)
    H = rng.integers(0, 50, size=(100, 150)).astype(np.int32)
    Ht = torch.from_numpy(H).to(dev)
    org = torch.tensor([[0, 0], [64, 100], [90, 140]], dtype=torch.int32, device=dev)
    tiles = fh.fh_tiles(Ht, org).float().cpu().numpy()
    mu = H.mean(axis=1)
    sd = H.std(axis=1)
    for t, (r0, c0) in enumerate([(0, 0), (64, 100), (90, 140)]):
        ref = np.zeros((64, 64))
        for y in range(64):
            for x in range(64):
                r, c = r0 + y, c0 + x
                if r < 100 and c < 150:
                    ref[y, x] = (H[r, c] - mu[r]) / sd[r]
        assert np.max(np.abs(tiles[t] - ref)) <= 2 ** -7 * np.max(np.abs(ref)) + 1e-6


def test_propose_ranks_tiles_by_score(dev):
    import torch
    from paper_1810_09784_amd import fh, synth
    from oracle import cnn as N
    rng = np.random.default_rng(7)
    spec = synth.cfg_single_small()
    pm = synth.make_peakmap(spec)
    plan = fh.Plan.from_spec(spec)
    H = fh.fh_hough(plan, torch.from_numpy(pm.row_ptr).to(dev), torch.from_numpy(pm.bin).to(dev))
    net = fh.CNN(max_batch=8)
    net.set_params(N.init_params(rng))
    scores, ids = fh.fh_propose(net, plan, H, 3)
    sc = scores.cpu().numpy()
    assert sc.shape == (12,)  # 2 x 6 tiles of 64 x 64 over the 128 x 323 map
    assert ids == list(np.argsort(-sc, kind="stable")[:3])
    # the same tiles through fh_tiles + forward give the same scores
    org = torch.tensor([[64 * (i // 6), 64 * (i % 6)] for i in range(12)], dtype=torch.int32, device=dev)
    tiles = fh.fh_tiles(H, org)
    # max_batch 8 < 12 tiles: fh_propose scores in pieces, so does this check
    lg = np.concatenate([net.forward(tiles[i:i + 8].contiguous()).cpu().numpy() for i in (0, 8)])
    assert np.allclose(lg, sc, rtol=0, atol=1e-6)
