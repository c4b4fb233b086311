"""The request server's micro-batch choice (host code in admission.hpp,
compiled with g++ under AddressSanitizer and UndefinedBehaviorSanitizer):
for seeded random queues, the indices each rule takes equal those of the
rule as stated, written out here independently, and satisfy its invariants
(the oldest request always taken, arrival order, the size limits, no closer
dataset left out of a full ragged batch)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("admission") / "admission_driver")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "paper_1203_1269_amd", "csrc"),
                           os.path.join(ROOT, "tests", "admission_driver.cpp"), "-o", exe])
    return exe


def expected_dataset(ds, max_batch):
    """Per-dataset rule: the oldest request's dataset, up to max_batch of its
    requests in arrival order."""
    if not ds or max_batch <= 0:
        return []
    return [q for q, k in enumerate(ds) if k == ds[0]][:max_batch]


def expected_ragged(ds, order, max_batch, max_datasets):
    """Ragged rule: the oldest request's dataset, then the other queued
    datasets by distance of their order from its order (ties: the dataset
    whose oldest queued request came first), max_datasets in all; their
    requests in arrival order, up to max_batch."""
    if not ds or max_batch <= 0 or max_datasets <= 0:
        return []
    first = {}
    for q, k in enumerate(ds):
        first.setdefault(k, q)
    k0 = ds[0]
    others = sorted((k for k in first if k != k0),
                    key=lambda k: (abs(order[k] - order[k0]), first[k]))
    chosen = set([k0] + others[:max_datasets - 1])
    return [q for q, k in enumerate(ds) if k in chosen][:max_batch]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_admission_rules(driver, seed):
    r = subprocess.run([driver, str(seed)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.strip().splitlines()
    assert len(lines) == 800
    for line in lines:
        head, qs, os_, tk = line.split(":")
        rule, queued, max_batch, max_datasets = head.split()
        ds = [int(x) for x in qs.split()]
        order = [int(x) for x in os_.split()]
        taken = [int(x) for x in tk.split()]
        assert len(ds) == int(queued)
        mb, md = int(max_batch), int(max_datasets)
        if rule == "D":
            assert taken == expected_dataset(ds, mb), line
            assert len({ds[q] for q in taken}) <= 1
        else:
            assert taken == expected_ragged(ds, order, mb, md), line
            assert len({ds[q] for q in taken}) <= md
            # no dataset left out is closer in order to the oldest request's
            # than a chosen one
            if taken:
                n0 = order[ds[0]]
                got = {ds[q] for q in taken}
                if len(got) == md:
                    far = max(abs(order[k] - n0) for k in got)
                    assert all(abs(order[k] - n0) >= far for k in set(ds) - got)
        # invariants of both rules
        assert taken == sorted(set(taken))
        assert len(taken) <= max(mb, 0)
        if ds and mb > 0 and (rule == "D" or md > 0):
            assert taken[0] == 0   # the oldest request is always taken
