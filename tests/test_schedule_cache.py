"""Schedule cache of the batched launch and the mix signature (host only).

The cache maps (GPU architecture name, compute units, mix signature) to a
tuned schedule in one JSON file; these tests drive the library's reader and
writer through the C ABI without a GPU."""
import json
import os

import pytest

import mtp_workloads as W
import paper_2505_01059_amd as mtp
from paper_2505_01059_amd._native import MtpError

ARCH = "gfx950:sramecc+:xnack-"
SCHED = {"wg_per_cu": 1, "order": 0, "cand_tiles": 2, "roll_tiles": 4, "refit_outputs": 16, "split_pct": 25}


def _mix():
    return [W.point_mass_config(name="s_pm", n_tensor=300, n_gauss=45, horizon=37, n_elites=20, n_iters=3, seed=1),
            W.chain_config(name="s_c7", n_tensor=700, n_gauss=101, horizon=66, n_elites=40, n_iters=2, seed=2)]


def test_store_then_lookup_round_trip(tmp_path):
    path = str(tmp_path / "sched.json")
    assert mtp.schedule_cache_lookup(path, ARCH, 256, 0x1234) is None     # no file yet
    mtp.schedule_cache_store(path, ARCH, 256, 0x1234, SCHED, 87.5)
    got = mtp.schedule_cache_lookup(path, ARCH, 256, 0x1234)
    assert got is not None
    sched, ms = got
    assert sched == SCHED and ms == pytest.approx(87.5)
    doc = json.load(open(path))
    assert doc["format"] == "mtp-schedules-1"
    (e,) = doc["entries"]
    assert e["arch"] == ARCH and e["cus"] == 256 and e["mix"] == "0000000000001234"
    assert {k: e[k] for k in SCHED} == SCHED


def test_key_is_arch_cus_and_mix(tmp_path):
    path = str(tmp_path / "sched.json")
    mtp.schedule_cache_store(path, ARCH, 256, 7, SCHED, 1.0)
    assert mtp.schedule_cache_lookup(path, "gfx942:sramecc+:xnack-", 256, 7) is None
    assert mtp.schedule_cache_lookup(path, ARCH, 304, 7) is None
    assert mtp.schedule_cache_lookup(path, ARCH, 256, 8) is None
    assert mtp.schedule_cache_lookup(path, ARCH, 256, 7) is not None


def test_store_replaces_its_key_and_keeps_the_others(tmp_path):
    path = str(tmp_path / "sched.json")
    other = dict(SCHED, cand_tiles=4, split_pct=0)
    mtp.schedule_cache_store(path, ARCH, 256, 1, SCHED, 2.0)
    mtp.schedule_cache_store(path, ARCH, 256, 2, other, 3.0)
    newer = dict(SCHED, refit_outputs=64)
    mtp.schedule_cache_store(path, ARCH, 256, 1, newer, 1.5)
    assert mtp.schedule_cache_lookup(path, ARCH, 256, 1) == (newer, 1.5)
    assert mtp.schedule_cache_lookup(path, ARCH, 256, 2) == (other, 3.0)
    assert len(json.load(open(path))["entries"]) == 2
    assert not [f for f in os.listdir(tmp_path) if ".tmp." in f]        # the temporary was renamed


@pytest.mark.parametrize("text", ["{not json", '{"format": "something-else", "entries": []}',
                                  '{"format": "mtp-schedules-1", "entries": [{"arch": "x"}]}', "[]"])
def test_a_file_that_is_not_a_cache_is_never_overwritten(tmp_path, text):
    path = tmp_path / "sched.json"
    path.write_text(text)
    assert mtp.schedule_cache_lookup(str(path), ARCH, 256, 1) is None
    with pytest.raises(MtpError):
        mtp.schedule_cache_store(str(path), ARCH, 256, 1, SCHED, 1.0)
    assert path.read_text() == text


@pytest.mark.parametrize("bad", [dict(cand_tiles=3), dict(roll_tiles=8), dict(refit_outputs=2),
                                 dict(refit_outputs=128), dict(order=2), dict(wg_per_cu=-1), dict(split_pct=-5)])
def test_store_rejects_schedules_the_kernel_does_not_support(tmp_path, bad):
    path = str(tmp_path / "sched.json")
    with pytest.raises(MtpError):
        mtp.schedule_cache_store(path, ARCH, 256, 1, dict(SCHED, **bad), 1.0)
    assert not os.path.exists(path)


def test_entries_with_unsupported_values_are_not_returned(tmp_path):
    path = tmp_path / "sched.json"
    entry = dict(arch=ARCH, cus=256, mix="0000000000000001", ms=1.0, **dict(SCHED, cand_tiles=3))
    path.write_text(json.dumps({"format": "mtp-schedules-1", "entries": [entry]}))
    assert mtp.schedule_cache_lookup(str(path), ARCH, 256, 1) is None


def test_mix_signature_follows_the_shapes_only():
    base = _mix()
    sig = mtp.mix_signature(base)
    assert sig != 0 and sig == mtp.mix_signature(_mix())
    # seeds and float parameters do not enter
    assert mtp.mix_signature([base[0].replace(seed=99), base[1].replace(temperature=3.0)]) == sig
    # shapes and the order of the instances do
    assert mtp.mix_signature([base[0].replace(horizon=38), base[1]]) != sig
    assert mtp.mix_signature([base[0], base[1].replace(n_tensor=701)]) != sig
    assert mtp.mix_signature([base[0], base[1].replace(n_iters=3)]) != sig
    assert mtp.mix_signature(base[::-1]) != sig
    assert mtp.mix_signature(base[:1]) != sig
