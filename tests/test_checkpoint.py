"""Checkpoints: parameters, model description and seeds in an .npz file
that loads without unpickling, bitwise round trip (CPU)."""

import dataclasses

import numpy as np

from mpinputs import ModelSpec, init_params
from paper_2410_01657_amd.model import load_checkpoint, save_checkpoint


def test_checkpoint_round_trip(tmp_path):
    spec = ModelSpec(H=64, n_layers=4, layernorm=True)
    params = init_params(spec, seed=11, perturb=True)
    path = tmp_path / "model.npz"
    save_checkpoint(path, params, spec, seed=11, step=0, lr=0.002)
    back, spec_fields, meta = load_checkpoint(path)
    assert sorted(back) == sorted(params)
    for k, v in params.items():
        assert back[k].dtype == np.float32 and back[k].shape == v.shape
        assert np.array_equal(back[k].view(np.uint32), v.view(np.uint32)), k
    assert ModelSpec(**spec_fields) == spec
    assert spec_fields == dataclasses.asdict(spec)
    assert meta == {"seed": 11, "step": 0, "lr": 0.002}
    # every entry is a plain numeric array: the file needs no pickle
    with np.load(path, allow_pickle=False) as z:
        assert all(z[k].dtype != object for k in z.files)


def test_checkpoint_regenerates_from_seed(tmp_path):
    # a checkpoint that records the seed reproduces the initial parameters
    spec = ModelSpec(H=32, n_layers=2, n_hidden=1)
    path = tmp_path / "init.npz"
    save_checkpoint(path, init_params(spec, seed=3), spec, seed=3)
    back, spec_fields, meta = load_checkpoint(path)
    again = init_params(ModelSpec(**spec_fields), seed=meta["seed"])
    assert all(np.array_equal(back[k], again[k]) for k in again)
