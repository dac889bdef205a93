"""Random-DAG workload: determinism, structure, and inherent sensitivity."""

import numpy as np
import pytest

from oracle.pyoracle import Program as OProg
from workloads import inputs
from workloads.rdag import rdag


def test_seeded_and_deterministic():
    assert rdag(1).text() == rdag(1).text()
    assert rdag(1).text() != rdag(2).text()


def test_structure_of_config_dag():
    p, st = rdag(1, 8, 200, return_stats=True)
    assert st["drawn"] == 200 and st["width"] == 17
    assert p.nnz_in == [8] and p.nnz_out == [4]
    c = p.op_counts()
    assert c["OUTPUT"] == 4 and c["INPUT"] <= 8
    # guards are primitive instructions: DIVG adds FABS+ADD, EXPG FMIN+FMAX, SQRTG FABS+ADD
    assert st["emitted"] >= 200
    assert set(c) <= {"INPUT", "OUTPUT", "CONST", "ADD", "SUB", "MUL", "DIV", "SIN", "COS",
                      "EXP", "SQRT", "TANH", "FABS", "FMIN", "FMAX"}


def _err(y, r):
    sc = np.sqrt(np.mean(r ** 2, axis=1, keepdims=True))
    sc[sc == 0] = 1
    return np.max(np.abs(y - r) / np.maximum(np.abs(r), sc))


def test_inherent_sensitivity_and_bounds(tmp_path):
    p = rdag(1, 8, 200)
    path = tmp_path / "r.xgp"
    p.save(path)
    o = OProg(path)
    x = inputs.uniform(101, 8, 1000)
    y64 = o.evaluate([x], 64)[0]
    y80 = o.evaluate([x], 80)[0]
    assert np.all(np.isfinite(y64)) and np.max(np.abs(y64)) <= 1e6
    assert _err(y64, y80) <= 1e-13


@pytest.mark.slow
@pytest.mark.parametrize("seed,n_in,n_ops", [(51, 16, 1000), (52, 32, 10000), (53, 64, 100000)])
def test_batch_dags_fp32_inherent_error(tmp_path, seed, n_in, n_ops):
    p = rdag(seed, n_in, n_ops, dtype="f32")
    path = tmp_path / "r.xgp"
    p.save(path)
    o = OProg(path)
    x = inputs.uniform(seed + 100, n_in, 256).astype(np.float32).astype(np.float64)
    y32 = o.evaluate([x], 32, threads=8)[0]
    y64 = o.evaluate([x], 64, threads=8)[0]
    y80 = o.evaluate([x], 80, threads=8)[0]
    assert np.all(np.isfinite(y64))
    assert _err(y64, y80) <= 1e-13
    assert _err(y32, y64) <= 2e-6
