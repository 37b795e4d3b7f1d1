"""The network's model-file reader (amg_mpnn_read_params), host only: the
committed JSON model files give the parameters the Python module stores in
them, a plain list of numbers is read as well, and unreadable or short files
are refused with AMG_ERR_MODEL."""
import json

import numpy as np
import pytest

import paper_2303_02352_amd as amd
from paper_2303_02352_amd import surrogate


@pytest.mark.parametrize("path", [surrogate.DEFAULT_MODEL, surrogate.RELAX640_MODEL])
def test_json_model_files(path):
    got = amd.read_model_params(path)
    ref = np.asarray(json.load(open(path))["params"], dtype=np.float32)
    assert got.shape == (amd.AMG_MPNN_NPARAMS,)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_plain_number_list(tmp_path):
    theta = np.random.default_rng(3).standard_normal(amd.AMG_MPNN_NPARAMS).astype(np.float32)
    f = tmp_path / "theta.txt"
    # eight per line, mixed separators; repr of a float32 widened to double reads back exactly
    lines = [", ".join(repr(float(x)) for x in theta[i:i + 8]) for i in range(0, theta.size, 8)]
    f.write_text("\n".join(lines) + "\n")
    got = amd.read_model_params(f)
    assert np.array_equal(got.view(np.uint32), theta.view(np.uint32))


@pytest.mark.parametrize("content", ["", "1 2 3", '{"params": [1.0, 2.0]}', '{"params": 5}',
                                     '{"params": [1.0, x]}'])
def test_unusable_files_are_refused(tmp_path, content):
    f = tmp_path / "bad.json"
    f.write_text(content)
    with pytest.raises(amd.AMGError) as e:
        amd.read_model_params(f)
    assert e.value.code == amd.AMG_ERR_MODEL


def test_missing_file_is_refused(tmp_path):
    with pytest.raises(amd.AMGError) as e:
        amd.read_model_params(tmp_path / "none.json")
    assert e.value.code == amd.AMG_ERR_MODEL
