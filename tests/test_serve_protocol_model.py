"""The served likelihood's slot protocol, modelled on the host with threads
(tests/serve_model/serve_protocol.cpp: the same claim, limit, done and fin
words and rules as the device loop) and run under ThreadSanitizer:

  * random traffic, the three claim policies, several slot and worker counts:
    every item processed once, every request completed once with its sum,
    no data race on the descriptors, partials or results;
  * a forced late claim: a worker that chose a slot while its request was
    finishing claims only after the next request was opened in the same
    slot; its claim is a valid item of the new request and nothing is lost;
  * the earlier claim rule (validate against the sequence number seen before
    the fetch_add), built with -DOLD_PROTOCOL, loses that item and stalls.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "serve_model", "serve_protocol.cpp")
ENV = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")


def _build(tmp_path, name, extra=()):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path / name)
    subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=thread", *extra, SRC, "-o", out],
                   check=True)
    return out


@pytest.fixture(scope="module")
def model_bin(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("serve_model"), "serve_protocol")


@pytest.mark.parametrize("policy", [0, 1, 2])
@pytest.mark.parametrize("workers,slots,seed", [(4, 4, 1), (7, 2, 2), (3, 16, 3), (12, 64, 4)])
def test_random_traffic_under_tsan(model_bin, policy, workers, slots, seed):
    r = subprocess.run([model_bin, "stress", str(policy), "200", str(workers), str(slots), str(seed)],
                       capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ThreadSanitizer" not in r.stderr


@pytest.mark.parametrize("policy", [0, 1, 2])
def test_late_claim_lands_on_the_next_request(model_bin, policy):
    r = subprocess.run([model_bin, "late", str(policy)], capture_output=True, text=True, env=ENV, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr


def test_old_claim_rule_loses_the_item(tmp_path):
    old = _build(tmp_path, "serve_protocol_old", ("-DOLD_PROTOCOL",))
    r = subprocess.run([old, "late", "1"], capture_output=True, text=True, env=ENV, timeout=120)
    assert r.returncode == 3, r.stdout + r.stderr
    assert "stalled" in r.stderr
