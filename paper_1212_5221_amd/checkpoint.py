"""Checkpoint and resume of a GaugeFixer's state through files.

A checkpoint is a directory with one ``inst<k>.npy`` per instance (the links
in the natural FP64-18 layout, as ``GaugeFixer.download`` returns them) and
``state.json``: lattice shapes, gauge, storage and, per instance, the global
sweep index that counts the random streams of the heatbath, stochastic
relaxation and annealing sweeps.  The random numbers depend only on the seed,
the instance, the sweep index and the site, so a run resumed from a
checkpoint continues the interrupted run exactly (the links of mixed storage
are stored in FP32 on the device, so their download and upload are exact).

The files are plain ``.npy`` arrays (loaded with ``allow_pickle=False``) and
JSON; nothing in a checkpoint is executed.
"""
from __future__ import annotations

import json
import os

import numpy as np

FORMAT = "gf-checkpoint-1"


def save(fx, path: str, extra: dict | None = None) -> None:
    """Write the links and sweep indices of every instance of `fx` to `path`."""
    os.makedirs(path, exist_ok=True)
    state = {"format": FORMAT, "dims": [list(d) for d in fx.dims], "group": int(fx.nc), "gauge": int(fx.gauge),
             "storage": int(fx.storage), "sweep_index": [], "extra": extra or {}}
    for k in range(len(fx.dims)):
        np.save(os.path.join(path, "inst%d.npy" % k), fx.download(k), allow_pickle=False)
        state["sweep_index"].append(int(fx.get_sweep_index(k)))
    with open(os.path.join(path, "state.json"), "w") as f:
        json.dump(state, f, indent=1)


def load(fx, path: str) -> dict:
    """Upload a checkpoint written by `save` into `fx`, which must have the same
    lattice shapes, gauge group, gauge and storage; returns the checkpoint's `extra`.
    Raises ValueError (nothing uploaded) on any mismatch."""
    with open(os.path.join(path, "state.json")) as f:
        state = json.load(f)
    if state.get("format") != FORMAT:
        raise ValueError("not a gauge-fixing checkpoint: %s" % path)
    if [tuple(d) for d in state["dims"]] != list(fx.dims):
        raise ValueError("lattice shapes differ: checkpoint %s, handle %s" % (state["dims"], fx.dims))
    if state.get("group", 3) != fx.nc or state["gauge"] != fx.gauge or state["storage"] != fx.storage:
        raise ValueError("gauge group, gauge or storage differ from the checkpoint's")
    links = []
    for k, d in enumerate(fx.dims):
        U = np.load(os.path.join(path, "inst%d.npy" % k), allow_pickle=False)
        want = (int(np.prod(d)), 4, fx.nc, fx.nc, 2)
        if U.shape != want or U.dtype != np.float64:
            raise ValueError("inst%d.npy holds %s %s, expected float64 %s" % (k, U.dtype, U.shape, want))
        links.append(U)
    # every file is read and checked before the first upload
    for k, U in enumerate(links):
        fx.upload(k, U)
        fx.set_sweep_index(k, state["sweep_index"][k])
    return state.get("extra", {})
