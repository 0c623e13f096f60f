"""The parity bar itself, on the CPU: an oracle run with float-level noise
injected stands in for the device.  Such a run must pass the bar (it is one
more correct result at float resolution), and runs with a mistake planted in
the oracle must fail it: one Gauss-Newton iteration too few, a Huber
threshold 2 % off, the depth-only Jacobian, and a 0.1 % inverse-depth bias
confined to the surfels the probe calls unstable (the case the per-surfel
cost bound is there for).  The damped variant on 5 px discs, where most
acceptance tests are near-ties, must pass as well."""
import dataclasses

import numpy as np
import pytest

import oracle
from scenegen import make_keyframe, spec_for_config
from scenegen.discs import make_disc_surfels
from tests.parity import as_dev, assert_parity, check_parity, oracle_keyframe, run_oracle_k, unstable_set


class HostKeyframe:
    """The attributes of a device keyframe that the parity helpers read."""

    def __init__(self, kf):
        self.K, self.R, self.t, self.patch = kf.K, kf.R, kf.t, kf.patch
        self._kf, self._nb = kf.kf_image.numpy(), kf.nbr_images.numpy()

    def dequantized_images(self):
        return self._kf, self._nb


def _noisy_run(hk, init_id, init_n, is_new, prm, seed, disc=None):
    """An oracle run with float-level noise (seeds outside the probe's),
    returned in the device's float32 layout."""
    st = run_oracle_k(oracle_keyframe(hk), init_id, init_n, is_new,
                      dataclasses.replace(prm, perturb=2e-6, perturb_seed=seed), disc=disc)
    d = as_dev(st)
    d["inv_depth"] = d["inv_depth"].astype(np.float32)
    d["n"] = d["n"].astype(np.float32)
    return d


@pytest.fixture(scope="module")
def small():
    spec = dataclasses.replace(spec_for_config(0), patch=4, n_nbr=3, half_new=True, seed=7)
    kf = make_keyframe(spec)
    return HostKeyframe(kf), kf, oracle.OracleParams(iters=spec.iters)


@pytest.mark.parametrize("seed", [77, 78])
def test_a_noisy_oracle_run_passes(small, seed):
    hk, kf, prm = small
    dev = _noisy_run(hk, kf.init_id, kf.init_n, kf.is_new, prm, seed)
    res = check_parity(hk, dev, kf.init_id, kf.init_n, kf.is_new, prm, label=f"noisy {seed}")
    assert_parity(res, label=f"noisy {seed}", max_unstable=0.13)
    # the classification is not a blanket exemption: most surfels are stable
    assert res.probe_unstable < 0.13 and res.within_all > 0.9


@pytest.mark.parametrize("mistake", ["one iteration less", "huber k +2%", "depth-only"])
def test_planted_mistakes_fail(small, mistake):
    hk, kf, prm = small
    bad = {"one iteration less": dataclasses.replace(prm, iters=prm.iters - 1),
           "huber k +2%": dataclasses.replace(prm, huber_k=prm.huber_k * 1.02),
           "depth-only": dataclasses.replace(prm, depth_only=True)}[mistake]
    dev = _noisy_run(hk, kf.init_id, kf.init_n, kf.is_new, bad, 77)
    res = check_parity(hk, dev, kf.init_id, kf.init_n, kf.is_new, prm, label=mistake)
    with pytest.raises(AssertionError):
        assert_parity(res, label=mistake, max_unstable=0.13)
    # the cost bound alone catches each of them as well
    assert res.cost_violations > 1


def test_a_bias_on_unstable_surfels_only_fails(small):
    hk, kf, prm = small
    okf = oracle_keyframe(hk)
    base = run_oracle_k(okf, kf.init_id, kf.init_n, kf.is_new, prm)
    uns, _ = unstable_set(hk, kf.init_id, kf.init_n, kf.is_new, prm, base)
    assert 0 < uns.mean() < 0.13
    dev = _noisy_run(hk, kf.init_id, kf.init_n, kf.is_new, prm, 77)
    dev["inv_depth"][uns] *= np.float32(1.001)
    res = check_parity(hk, dev, kf.init_id, kf.init_n, kf.is_new, prm, label="biased unstable")
    with pytest.raises(AssertionError, match="worst oracle outcome"):
        assert_parity(res, label="biased unstable", max_unstable=0.13)


def test_damped_variant_on_small_discs_passes():
    spec = dataclasses.replace(spec_for_config(1), width=320, height=240, n_nbr=4, n_rects=8, seed=62,
                               half_new=False)
    kf = make_keyframe(spec)
    d = make_disc_surfels(kf, radius=5.0)
    hk = HostKeyframe(kf)
    prm = oracle.OracleParams(iters=8, lm_lambda=1e-3)
    disc = (d.ux, d.uy, 5.0)
    dev = _noisy_run(hk, d.init_id, d.init_n, None, prm, 77, disc=disc)
    res = check_parity(hk, dev, d.init_id, d.init_n, None, prm, label="disc r5 LM noisy", disc=disc)
    assert_parity(res, label="disc r5 LM noisy", max_unstable=0.23)
