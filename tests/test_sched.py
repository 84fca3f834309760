"""Host scheduling of the server (admission, FIFO order, memory budget,
mid-flight admission, pass batching) on the CPU with a fake executor: the
scheduler header is compiled with g++ into a driver whose "solves" sleep.
The fake executor only schedules; it is never a compute path."""
import json
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sched") / "sched_fake")
    subprocess.run(["g++", "-O1", "-std=c++17", "-pthread", "-Wall", "-Wextra", "-o", exe,
                    os.path.join(HERE, "sched_fake.cpp")], check=True)
    return exe


def run(driver, which):
    out = subprocess.run([driver, which], check=True, capture_output=True, text=True, timeout=60)
    return json.loads(out.stdout)


def test_memory_budget_and_fifo(driver):
    r = run(driver, "budget")
    t = {x["id"]: x for x in r["tickets"]}
    a, b, c = (t[i] for i in r["ids"])
    # never two 60s at once; peak within the budget
    assert b["start"] >= a["end"] - 1e-4
    assert r["stats"]["peak_used"] <= 100
    # the 30 does not overtake the queued 60 (it would have fit beside the first)
    assert c["start"] >= b["start"] - 1e-4
    assert [x["status"] for x in (a, b, c)] == [0, 0, 0]
    assert r["stats"]["completed"] == 3
    # the idle workspaces (60 and 30) stay charged until shutdown
    assert r["stats"]["used"] == 90 and r["used_after_shutdown"] == 0
    # the second 60 ran on the slot whose workspace already held 60
    assert b["slot"] == a["slot"]


def test_idle_workspaces_are_charged(driver):
    """A slot's workspace stays charged after its request ends; an idle
    workspace is given back only when no idle slot can take the head request
    as things are; what the executors really hold never exceeds the budget."""
    r = run(driver, "resident")
    a, b, c, d = r["tickets"]
    assert [x["status"] for x in r["tickets"]] == [0, 0, 0, 0]
    assert c["slot"] == a["slot"]            # the idle 60 took the next 60
    assert r["stats"]["releases"] >= 1 and r["exec_releases"] == r["stats"]["releases"]
    assert r["stats"]["peak_used"] <= 100
    assert r["resident_peak"] <= 100
    # held workspaces are still charged when the last request has ended
    assert r["stats"]["used"] > 0
    assert r["used_after_shutdown"] == 0 and r["resident_after_shutdown"] == 0


def test_no_overcommit_with_resident_workspaces(driver):
    r = run(driver, "overcommit")
    assert all(x["status"] == 0 for x in r["tickets"])
    assert r["stats"]["completed"] == 5
    assert r["resident_peak"] <= 100 and r["stats"]["peak_used"] <= 100


def test_rejects_what_can_never_fit(driver):
    r = run(driver, "reject")
    assert r["ids"][0] == -1 and r["ids"][1] > 0
    assert "budget is 100" in r["rejected_msg"]
    assert r["stats"]["submitted"] == 1 and r["stats"]["completed"] == 1


def test_admitted_mid_flight(driver):
    r = run(driver, "midflight")
    t = r["tickets"]
    long, short = t[0], t[1:]
    # every short request started and finished while the long one ran
    assert all(s["start"] < long["end"] and s["end"] < long["end"] for s in short)
    assert r["stats"]["admitted_while_busy"] >= 3
    assert r["stats"]["peak_active"] == 2
    # executors are made once per slot, not per request
    assert r["executors"] == 2


def test_failure_is_per_request(driver):
    r = run(driver, "failure")
    assert [x["status"] for x in r["tickets"]] == [4, 0]


def test_shutdown_drains(driver):
    r = run(driver, "drain")
    assert r["stats"]["completed"] == 7 and r["stats"]["peak_active"] == 3


def test_batcher_packs_concurrent_posts(driver):
    r = run(driver, "batcher")
    assert r["every_job_once"] == 1 and r["seen"] == r["jobs"] == 120
    assert r["max_batch"] >= 2 and r["batches"] < 120


def test_batcher_window_gathers_staggered_posts(driver):
    """With a window, posts 20 ms apart wait for each other (one batch of
    three); without one, each runs as it comes."""
    r = run(driver, "window")
    assert r["every_job_once"] == 1 and r["batches"] == 1 and r["max_batch"] == 3
    r = run(driver, "nowindow")
    assert r["every_job_once"] == 1 and r["batches"] == 3 and r["max_batch"] == 1
