"""Host tests of the training loop's robustness helpers (no GPU): the
checkpoint round trip (weights, Adam state, step, generator), the
write-then-rename of checkpoint files, and the non-finite step guard."""
import math
import os

import numpy as np
import pytest
import torch

from paper_2512_21180_amd import learned, train


def _net():
    return learned.PDNet(n_iter=2, seed=3, scales=[2, 1], init="fdk")


def test_checkpoint_round_trip(tmp_path):
    net = _net()
    opt = torch.optim.Adam(net.parameters(), lr=1e-3)
    for k in range(2):   # give Adam non-trivial moments
        for p in net.parameters():
            p.grad = torch.full_like(p, 0.1 * (k + 1))
        opt.step()
    rng = np.random.default_rng(5)
    rng.random(7)
    path = str(tmp_path / "run.pt.ckpt")
    train.save_checkpoint(path, net, opt, 42, rng, 3)
    assert not os.path.exists(path + ".tmp")
    net2, opt_state, step, rng2, skipped = train.load_checkpoint(path, device="cpu")
    assert step == 42 and skipped == 3
    for (k, a), (k2, b) in zip(net.state_dict().items(), net2.state_dict().items()):
        assert k == k2 and torch.equal(a, b)
    assert net2.perms == net.perms and net2.scales == net.scales and net2.init == net.init
    opt2 = torch.optim.Adam(net2.parameters(), lr=1e-3)
    opt2.load_state_dict(opt_state)
    s1, s2 = opt.state_dict()["state"], opt2.state_dict()["state"]
    assert s1.keys() == s2.keys()
    for i in s1:
        assert torch.equal(s1[i]["exp_avg"], s2[i]["exp_avg"])
        assert torch.equal(s1[i]["exp_avg_sq"], s2[i]["exp_avg_sq"])
        assert float(s1[i]["step"]) == float(s2[i]["step"]) == 2.0
    # the generator continues the same sequence
    assert np.array_equal(rng.random(5), rng2.random(5))


def test_failed_write_keeps_previous_file(tmp_path):
    path = str(tmp_path / "w.pt")
    train.save(_net(), path, {})
    before = open(path, "rb").read()
    with pytest.raises(Exception):
        train._write({"bad": lambda v: v}, path)   # not serialisable
    assert open(path, "rb").read() == before
    assert train.load(path, device="cpu").n_iter == 2


def test_finite_step_guard():
    net = _net()
    ps = list(net.parameters())
    for p in ps:
        p.grad = torch.zeros_like(p)
    assert train.finite_step(0.5, ps)
    assert not train.finite_step(float("nan"), ps)
    assert not train.finite_step(math.inf, ps)
    ps[3].grad[0] = float("inf")
    assert not train.finite_step(0.5, ps)
    ps[3].grad[0] = float("nan")
    assert not train.finite_step(0.5, ps)


def test_committed_weights_load_on_host():
    here = os.path.dirname(os.path.abspath(train.__file__))
    net = train.load(os.path.join(here, "weights", "lpd_c5_multiscale_fdk.pt"), device="cpu")
    assert net.n_iter == 8 and net.scales == [4, 4, 4, 2, 2, 2, 1, 1] and net.init == "fdk"
