"""Run-time controls of the library (environment), through the C ABI:

* IM_TILE / IM_WAVES pick the leaf configuration with that tile size and
  workgroup size (the statistics report it), and results stay exact;
* a combination that matches no configuration is ignored;
* IM_AUTOTUNE_CACHE: an entry for this device's architecture and the call's
  workload class selects its configuration (entries of other architectures
  are skipped); the autotuner appends its choice to the file;
* IM_LOG=1 prints one plan line per merge call.
"""
import os
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2005_12648_amd as im

pytestmark = pytest.mark.gpu


def _merge_cfg(dev, data, la):
    t = torch.from_numpy(data).to(dev)
    im.inplace_merge(t, la)
    st = im.fetch_stats()
    assert np.array_equal(t.cpu().numpy(), oracle.merge(data, la))
    return st


def test_tile_and_waves_select_a_configuration(dev, monkeypatch):
    data, la = gen.make("c1")                      # int32
    monkeypatch.setenv("IM_TILE", str(256 * 35))
    monkeypatch.setenv("IM_WAVES", "4")
    st = _merge_cfg(dev, data, la)
    assert st["leaf_config"] == 2 and st["tile"] == 256 * 35
    monkeypatch.delenv("IM_TILE")
    monkeypatch.setenv("IM_WAVES", "4")            # first 4-wave configuration
    assert _merge_cfg(dev, data, la)["leaf_config"] == 2
    monkeypatch.setenv("IM_TILE", "12345")         # no such tile: ignored
    monkeypatch.delenv("IM_WAVES")
    assert _merge_cfg(dev, data, la)["leaf_config"] == 0


def test_autotune_cache_file(dev, monkeypatch, tmp_path):
    # a file the device has not read yet is read by its next merge
    arch = torch.cuda.get_device_properties(0).gcnArchName.replace(" ", "_")
    path = tmp_path / "tune.txt"
    data, la = gen.make("c1")
    n = data.size
    cls = 0
    while cls < 63 and (2 << cls) <= n:
        cls += 1
    path.write_text("# comment line, skipped\nimtune1 other_arch 4 0 %d 1\nimtune1 %s 4 0 %d 3\n"
                    % (cls, arch, cls))
    monkeypatch.setenv("IM_AUTOTUNE_CACHE", str(path))
    assert _merge_cfg(dev, data, la)["leaf_config"] == 3
    # the autotuner appends its choice
    inst, off = gen.batch(64, 77, 6.0, 14.0)
    t = torch.from_numpy(inst).to(dev)
    chosen, ms = im.autotune(t, torch.from_numpy(off).to(dev), reps=1)
    lines = path.read_text().strip().splitlines()
    assert lines[-1].split()[:3] == ["imtune1", arch, "4"]
    assert int(lines[-1].split()[-1]) == chosen
    assert np.array_equal(t.cpu().numpy(), inst)          # the autotuner leaves its input alone
    # forget the entry for the class of the merge above again (other tests)
    path.write_text("imtune1 %s 4 0 %d 0\n" % (arch, cls))
    monkeypatch.setenv("IM_AUTOTUNE_CACHE", str(tmp_path / "other"))
    (tmp_path / "other").write_text("imtune1 %s 4 0 %d 0\n" % (arch, cls))
    assert _merge_cfg(dev, data, la)["leaf_config"] == 0


def test_log_prints_the_plan(dev, monkeypatch, capfd):
    monkeypatch.setenv("IM_LOG", "1")
    data, la = gen.make("c1")
    _merge_cfg(dev, data, la)
    err = capfd.readouterr().err
    assert "[inplace_merge]" in err and "leaf config" in err and "level(s) enqueued" in err
