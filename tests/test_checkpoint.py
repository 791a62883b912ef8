"""Checkpoint files: host logic only (a stand-in handle keeps the links in host
memory; the GPU test of a resumed anneal is in test_gpu_anneal.py)."""
import json
import os

import numpy as np
import pytest

from paper_1212_5221_amd import checkpoint


class HostFixer:
    """Holds what save/load touch on a GaugeFixer: shapes, gauge, storage,
    links per instance and the per-instance sweep index."""

    def __init__(self, dims, gauge=0, storage=2, nc=3):
        self.dims = [tuple(d) for d in dims]
        self.nc = nc
        self.gauge = gauge
        self.storage = storage
        self.links = [np.zeros((int(np.prod(d)), 4, nc, nc, 2)) for d in self.dims]
        self.index = [0] * len(self.dims)

    def download(self, k):
        return self.links[k].copy()

    def upload(self, k, U):
        assert U.shape == self.links[k].shape and U.dtype == np.float64
        self.links[k] = U.copy()

    def get_sweep_index(self, k):
        return self.index[k]

    def set_sweep_index(self, k, i):
        self.index[k] = i


def _filled(dims, seed):
    fx = HostFixer(dims)
    rng = np.random.default_rng(seed)
    for k in range(len(dims)):
        fx.links[k] = rng.standard_normal(fx.links[k].shape)
        fx.index[k] = int(rng.integers(0, 1 << 40))
    return fx


def test_round_trip_restores_links_and_sweep_indices(tmp_path):
    dims = [(2, 4, 2, 4), (4, 2, 2, 2)]
    a = _filled(dims, 1)
    checkpoint.save(a, str(tmp_path), extra={"T": 0.25, "step": 7})
    b = HostFixer(dims)
    assert checkpoint.load(b, str(tmp_path)) == {"T": 0.25, "step": 7}
    for k in range(len(dims)):
        np.testing.assert_array_equal(b.links[k], a.links[k])
        assert b.index[k] == a.index[k]


def test_files_are_plain_arrays_and_json(tmp_path):
    a = _filled([(2, 2, 2, 2)], 2)
    checkpoint.save(a, str(tmp_path))
    assert sorted(os.listdir(tmp_path)) == ["inst0.npy", "state.json"]
    with open(tmp_path / "state.json") as f:
        state = json.load(f)
    assert state["format"] == checkpoint.FORMAT and state["dims"] == [[2, 2, 2, 2]]
    np.testing.assert_array_equal(np.load(tmp_path / "inst0.npy", allow_pickle=False), a.links[0])


@pytest.mark.parametrize("change", ["dims", "count", "group", "gauge", "storage", "format", "array"])
def test_mismatches_are_refused_before_anything_is_uploaded(tmp_path, change):
    dims = [(2, 4, 2, 4), (2, 2, 2, 2)]
    a = _filled(dims, 3)
    checkpoint.save(a, str(tmp_path))
    b = HostFixer(dims)
    if change == "dims":
        b = HostFixer([(4, 2, 2, 4), (2, 2, 2, 2)])
    elif change == "count":
        b = HostFixer(dims[:1])
    elif change == "group":
        b = HostFixer(dims, nc=2)
    elif change == "gauge":
        b.gauge = 2
    elif change == "storage":
        b.storage = 0
    elif change == "array":
        np.save(tmp_path / "inst1.npy", np.zeros((16, 4, 3, 3, 2), np.float32), allow_pickle=False)
    else:
        with open(tmp_path / "state.json") as f:
            state = json.load(f)
        state["format"] = "something-else"
        with open(tmp_path / "state.json", "w") as f:
            json.dump(state, f)
    before = [x.copy() for x in b.links]
    with pytest.raises(ValueError):
        checkpoint.load(b, str(tmp_path))
    for x, y in zip(b.links, before):
        np.testing.assert_array_equal(x, y)
