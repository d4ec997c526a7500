"""The bench line's recorded update-kernel traffic and VALU count belong to the kernel source in
the tree: the bench reports them only while the source hash matches, so a stale record would
silently turn `roofline.traffic` into null.  These checks make such a record fail loudly, and
tie the numbers to the counter summary committed under profiles/."""
import hashlib
import importlib.util
import os
import re

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PROFILE = os.path.join(ROOT, "profiles", "c2_channel_traffic.md")


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _source_hash():
    path = os.path.join(ROOT, "paper_1810_08137_amd", "csrc", "ugks_kernels.hip")
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def _profile_rows():
    """kernel name -> (traffic GB, VALU wave instructions in millions) from the first table."""
    rows = {}
    with open(PROFILE) as fh:
        for line in fh:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) == 10 and cells[0].startswith(("update_kernel", "sums_kernel")):
                rows[cells[0]] = (float(cells[5]), float(cells[6].rstrip("M")))
    return rows


def test_recorded_traffic_is_for_the_kernel_source_in_the_tree():
    b = _bench()
    assert b.MEASURED_TRAFFIC["source_sha256"] == _source_hash(), (
        "the recorded update-kernel counters are for another kernel source: record them again")
    assert b.measured_traffic("fp64") is not None


def test_counter_summary_names_the_same_source():
    with open(PROFILE) as fh:
        text = fh.read()
    m = re.search(r"SHA-256 \(`paper_1810_08137_amd/csrc/ugks_kernels.hip`\): `([0-9a-f]{64})`", text)
    assert m, "the counter summary states no kernel source hash"
    assert m.group(1) == _source_hash()


@pytest.mark.parametrize("form,kernel", [("fp64", "update_kernel<double, 2>"),
                                         ("fp32_store", "update_kernel<float, 1>")])
def test_recorded_traffic_matches_the_counter_summary(form, kernel):
    b = _bench()
    rows = _profile_rows()
    assert kernel in rows, f"{kernel} missing from {PROFILE}"
    gb, _ = rows[kernel]
    assert abs(b.MEASURED_TRAFFIC[form] / 1e9 - gb) <= 5e-4


def test_recorded_valu_count_matches_the_counter_summary():
    b = _bench()
    _, valu_m = _profile_rows()["update_kernel<double, 2>"]
    assert abs(b.MEASURED_TRAFFIC["valu_fp64"] / 1e6 - valu_m) <= 0.01
