"""The stored oracle results under tests/golden match the generators that
rebuild their inputs: every case's geometry and seed in cK_golden.json equal
what make_cK_golden.case_config derives from synth today, and each stored
c_K has that configuration's shape, finite values and the recorded norm.
(A generator change that would silently make the GPU tests compare against
a different problem fails here, on the CPU.)"""
import importlib.util
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
_spec = importlib.util.spec_from_file_location("make_cK_golden",
                                               os.path.join(GOLDEN, "make_cK_golden.py"))
mk = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(mk)
TABLE = json.load(open(mk.JSON))
NAMES = sorted(k for k in TABLE if not k.startswith("_"))


@pytest.mark.parametrize("name", NAMES)
def test_stored_case_matches_generator(name):
    meta = TABLE[name]
    cfg, k1, k2 = mk.case_config(name)
    got = dict(side=cfg.nx, nz=cfg.nz, n_species=cfg.n_species, n_pulses=cfg.n_pulses,
               nt=cfg.nt, f=cfg.f, seed=cfg.seed, k1=k1, k2=k2)
    assert {k: meta[k] for k in got} == got
    c = np.load(os.path.join(GOLDEN, f"cK_{name}.npy"))
    assert c.shape == cfg.c_shape and c.dtype == np.float32
    assert np.isfinite(c).all() and (c >= 0).all()
    assert float(np.linalg.norm(c.astype(np.float64))) == pytest.approx(meta["norm_cK"], rel=1e-6)
    assert meta["alpha1"] == pytest.approx(1.0 / (1.01 * meta["eig_max"]), rel=1e-12)


def test_every_case_is_stored():
    assert set(mk.CASES) <= set(NAMES)
