"""Checkpoint and resume of the CNN training loop.  CPU: a stand-in network
whose update depends on the parameters, the optimiser state and the batch
order, so a resumed run equals an uninterrupted one only when all three are
restored.  GPU: the library's optimiser state round trip, and one Adam step
after a restore equal, bit for bit, to the step the saving network takes."""
import numpy as np
import pytest

from paper_1810_09784_amd import learn


class StandIn:
    """The network interface train() uses, with a deterministic numpy update."""

    def __init__(self):
        self.p = np.zeros(5, dtype=np.float32)
        self.m1 = np.zeros(5, dtype=np.float32)
        self.m2 = np.zeros(5, dtype=np.float32)
        self.steps = 0
        self.x = None

    def forward(self, X):
        self.x = X.numpy().astype(np.float32)

    def backward(self, y):
        import torch
        g = (self.x.mean(axis=0) - y.numpy().mean()) * (1 + self.p)
        self.g = g.astype(np.float32)
        return torch.tensor([float(np.square(g).sum())])

    def step(self, lr):
        self.steps += 1
        self.m1 = 0.9 * self.m1 + 0.1 * self.g
        self.m2 = 0.999 * self.m2 + 0.001 * self.g * self.g
        self.p = self.p - lr * self.m1 / (np.sqrt(self.m2) + 1e-3) / self.steps

    def get_params(self):
        return self.p.copy(), None

    def set_params(self, p):
        self.p = np.asarray(p, dtype=np.float32).copy()
        self.m1[:] = 0
        self.m2[:] = 0
        self.steps = 0

    def get_state(self):
        return self.m1.copy(), self.m2.copy(), self.steps

    def set_state(self, m1, m2, steps):
        self.m1, self.m2, self.steps = np.asarray(m1).copy(), np.asarray(m2).copy(), int(steps)


def _data():
    import torch
    g = torch.Generator().manual_seed(3)
    return torch.randn(40, 5, generator=g), (torch.rand(40, generator=g) > 0.5).float()


def test_resumed_training_equals_uninterrupted(tmp_path):
    X, y = _data()
    ref = StandIn()
    h_ref = learn.train(ref, X, y, epochs=4, lr=0.05, batch=8, seed=11)

    ck = str(tmp_path / "train.npz")

    class Stop(Exception):
        pass

    def stop_after_one(ep):
        if ep == 1:
            raise Stop()

    first = StandIn()
    with pytest.raises(Stop):
        learn.train(first, X, y, epochs=4, lr=0.05, batch=8, seed=11, checkpoint=ck, after_epoch=stop_after_one)
    resumed = StandIn()  # a fresh process: nothing but the checkpoint carries over
    h = learn.train(resumed, X, y, epochs=4, lr=0.05, batch=8, seed=11, checkpoint=ck)
    assert h == h_ref
    np.testing.assert_array_equal(resumed.p, ref.p)
    np.testing.assert_array_equal(resumed.m1, ref.m1)
    assert resumed.steps == ref.steps == 4 * 5
    # a finished run's checkpoint resumes to nothing more
    again = StandIn()
    assert learn.train(again, X, y, epochs=4, lr=0.05, batch=8, seed=11, checkpoint=ck) == h_ref
    np.testing.assert_array_equal(again.p, ref.p)


def test_checkpoint_of_another_run_is_refused(tmp_path):
    X, y = _data()
    ck = str(tmp_path / "train.npz")
    learn.train(StandIn(), X, y, epochs=1, lr=0.05, batch=8, seed=11, checkpoint=ck)
    for kw in (dict(seed=12), dict(batch=4), dict(lr=0.1)):
        args = dict(epochs=2, lr=0.05, batch=8, seed=11, checkpoint=ck)
        args.update(kw)
        with pytest.raises(ValueError):
            learn.train(StandIn(), X, y, **args)


@pytest.mark.gpu
def test_optimiser_state_restore_continues_bit_for_bit():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_09784_amd import fh
    from oracle import cnn as N
    rng = np.random.default_rng(5)
    p0 = N.init_params(rng).astype(np.float32)
    g1 = (rng.standard_normal(p0.size) * 1e-2).astype(np.float32)
    g2 = (rng.standard_normal(p0.size) * 1e-2).astype(np.float32)
    a = fh.CNN(max_batch=4)
    a.set_params(p0)
    a.set_grads(g1)
    a.step(1e-3)
    p1, _ = a.get_params()
    m1, m2, steps = a.get_state()
    assert steps == 1 and np.any(m1 != 0) and np.any(m2 != 0)
    a.set_grads(g2)
    a.step(1e-3)
    p2_a, _ = a.get_params()
    b = fh.CNN(max_batch=4)
    b.set_params(p1)
    b.set_state(m1, m2, steps)
    r1, r2, rs = b.get_state()
    np.testing.assert_array_equal(r1, m1)
    np.testing.assert_array_equal(r2, m2)
    assert rs == steps
    b.set_grads(g2)
    b.step(1e-3)
    p2_b, _ = b.get_params()
    np.testing.assert_array_equal(p2_b, p2_a)
    a.destroy()
    b.destroy()
