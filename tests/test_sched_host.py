"""The serving scheduler on the host (tina_server_schedule_simulate): the same
admission, per-step quota, cancellation and step-completion decisions the
running server makes, driven by a script instead of device work.  Runs
without a GPU (the library loads; the simulate call makes no HIP call)."""
import os
import shutil
import subprocess

import pytest

from paper_2408_16551_amd import pfb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def lib():
    if not os.path.exists(pfb.LIB_PATH):
        pytest.skip("libtina_pfb.so not built")
    return pfb.load()


def sim(ops, **kw):
    return pfb.schedule_simulate(ops, **kw)


def of(ev, kind):
    return [e for e in ev if e["kind"] == kind]


def step_items(ev):
    """Steps as lists of (id, samples, frames), split at the end markers."""
    steps, cur = [], []
    for e in ev:
        if e["kind"] != "step":
            continue
        if e["id"] == 0:
            steps.append(cur)
            cur = []
        else:
            cur.append((e["id"], e["a"], e["b"]))
    return steps


def test_admission_in_arrival_order_one_request_per_stream_and_slot_limit():
    P = 64
    ops = [("add_stream", P, 0), ("add_stream", P, 0), ("add_stream", P, 0)]
    ops += [("submit", 0, P * 10), ("submit", 0, P * 10), ("submit", 1, P * 10), ("submit", 2, P * 10)]
    ops += [("admit", 0, 0)]
    ev = sim(ops, max_active=2)
    # requests 1 (stream 0) and 3 (stream 1): request 2 waits for its stream, 4 for a slot
    assert [e["id"] for e in of(ev, "admit")] == [1, 3]


def test_request_that_does_not_fit_blocks_the_ones_behind_it():
    P = 64
    row = 8 * P
    big = 100 * P   # in 100 P * 8 bytes + out 100 rows
    arena = 8 * big + 100 * row + 4096
    ops = [("add_stream", P, 0), ("add_stream", P, 0), ("add_stream", P, 0)]
    ops += [("submit", 0, big), ("submit", 1, big), ("submit", 2, P)]
    ops += [("admit", 0, 0)]
    ev = sim(ops, max_active=8, arena_bytes=arena)
    assert [e["status"] for e in of(ev, "submit")] == [0, 0, 0]
    # the second big request does not fit while the first holds the arena: the
    # small third request waits behind it (no starvation of large requests)
    assert [e["id"] for e in of(ev, "admit")] == [1]
    ops += [("ready", 0, 1), ("step", 0, 0), ("complete", 0, 0), ("admit", 0, 0)]
    ev = sim(ops, max_active=8, arena_bytes=arena, frames_per_step=1000)
    assert [e["id"] for e in of(ev, "admit")] == [1, 2, 3]


def test_a_request_larger_than_the_budget_is_refused():
    ev = sim([("add_stream", 64, 0), ("submit", 0, 64 * 1000)], arena_bytes=64 * 1000 * 8)
    assert of(ev, "submit")[0]["status"] == 7  # TOO_LARGE: input plus output exceed the arena
    assert of(ev, "submit")[0]["id"] == 0


def test_queue_limit_returns_busy():
    ops = [("add_stream", 64, 0)] + [("submit", 0, 64)] * 3
    ev = sim(ops, max_queued=2)
    assert [e["status"] for e in of(ev, "submit")] == [0, 0, 5]


@pytest.mark.parametrize("n_ready", [1, 2, 3, 4, 8])
def test_per_step_quota_scales_with_the_free_slots(n_ready):
    P, fps, slots = 32, 16, 8
    ops = [("add_stream", P, 0) for _ in range(n_ready)]
    ops += [("submit", i, P * 1000, ) for i in range(n_ready)]
    ops += [("admit", 0, 0)] + [("ready", 0, i + 1) for i in range(n_ready)] + [("step", 0, 0)]
    steps = step_items(sim(ops, max_active=slots, frames_per_step=fps))
    quota = fps * max(1, slots // n_ready)
    assert len(steps) == 1 and len(steps[0]) == n_ready
    for _, samples, frames in steps[0]:
        assert frames == quota and samples == quota * P


def test_chunks_of_a_stream_continue_its_residue_and_complete_every_frame():
    P, fps = 16, 4
    sizes = [P * 7 + 5, 3, P * 2 + 9, 1]    # residues carry from request to request
    ops = [("add_stream", P, 0)] + [("submit", 0, n) for n in sizes]
    for rid in range(1, len(sizes) + 1):
        ops += [("admit", 0, 0), ("ready", 0, rid)]
        ops += [("step", 0, 0), ("complete", 0, 0)] * 4
    ev = sim(ops, max_active=1, frames_per_step=fps)
    done = {e["id"]: e for e in of(ev, "complete") if e["id"]}
    assert sorted(done) == [1, 2, 3, 4] and all(e["status"] == 0 for e in done.values())
    want = [e["b"] for e in of(ev, "submit")]
    assert [done[i]["a"] for i in range(1, 5)] == want
    assert sum(want) == sum(sizes) // P
    # every step respects the quota (one request, one slot: fps frames)
    for st in step_items(ev):
        for _, _, frames in st:
            assert frames <= fps


def test_cancel_newest_queued_only_and_not_an_admitted_request():
    P = 64
    ops = [("add_stream", P, 0), ("submit", 0, P * 4), ("submit", 0, P * 4), ("submit", 0, P * 4)]
    ops += [("admit", 0, 0), ("cancel", 0, 2), ("cancel", 0, 1), ("cancel", 0, 3), ("cancel", 0, 2)]
    ev = sim(ops, max_active=4)
    assert [e["status"] for e in of(ev, "cancel")] == [1, 6, 0, 0]
    # 2: not the newest queued of its stream; 1: already admitted; 3 then 2: newest first


def test_failed_step_ends_its_requests_and_the_others_continue():
    P = 32
    ops = [("add_stream", P, 0), ("add_stream", P, 0)]
    ops += [("submit", 0, P * 100), ("submit", 1, P * 100), ("submit", 0, P * 5)]
    ops += [("admit", 0, 0), ("ready", 0, 1), ("step", 0, 0), ("ready", 0, 2), ("step", 0, 0)]
    ops += [("complete", 4, 0)]           # the first step (request 1 only) fails with DEVICE
    ops += [("complete", 0, 0)] + [("step", 0, 0), ("complete", 0, 0)] * 10
    ops += [("admit", 0, 0), ("ready", 0, 3), ("step", 0, 0), ("complete", 0, 0)]
    ev = sim(ops, max_active=4, frames_per_step=16)
    done = {e["id"]: e for e in of(ev, "complete") if e["id"]}
    assert done[1]["status"] == 4
    assert done[2]["status"] == 0 and done[2]["a"] == 100
    # the failed request's stream takes its next request (residue continues from the issued steps)
    assert done[3]["status"] == 0
    # request 1's later steps are skipped once it failed
    assert all(item[0] != 1 for st in step_items(ev)[2:] for item in st)


def test_two_steps_in_flight_complete_in_order():
    P = 16
    ops = [("add_stream", P, 0), ("submit", 0, P * 40), ("admit", 0, 0), ("ready", 0, 1)]
    ops += [("step", 0, 0), ("step", 0, 0), ("complete", 0, 0)]
    ev = sim(ops, max_active=1, frames_per_step=20)
    assert not [e for e in of(ev, "complete") if e["id"] == 1]   # half its frames are still in flight
    ops += [("complete", 0, 0)]
    ev = sim(ops, max_active=1, frames_per_step=20)
    done = [e for e in of(ev, "complete") if e["id"] == 1]
    assert done and done[0]["a"] == 40 and done[0]["b"] == 2


def test_device_buffers_use_no_arena_and_are_ready_on_admission():
    P = 64
    ops = [("add_stream", P, 0), ("submit", 0, -P * 1000), ("admit", 0, 0), ("step", 0, 0), ("complete", 0, 0)]
    ev = sim(ops, max_active=1, frames_per_step=2000, arena_bytes=4096)
    assert of(ev, "admit")[0]["a"] == -1 and of(ev, "admit")[0]["b"] == -1
    assert [e for e in of(ev, "complete") if e["id"] == 1][0]["a"] == 1000


def test_empty_request_completes_without_a_step():
    ops = [("add_stream", 64, 0), ("submit", 0, 0), ("admit", 0, 0), ("ready", 0, 1), ("step", 0, 0)]
    ev = sim(ops)
    assert [e for e in of(ev, "complete") if e["id"] == 1][0]["status"] == 0
    assert step_items(ev) == [[]]


@pytest.mark.parametrize("sanitizer", ["address,undefined", "thread"])
def test_scheduler_under_sanitizers(sanitizer, tmp_path):
    """The scheduler source built for the host with g++ sanitizers, driven by
    randomised scenarios (tests/sched_driver.cpp): a submitter thread and a
    loop thread share it under a mutex, as in the server."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "sched_driver"
    cmd = [gxx, "-std=c++17", "-O1", "-g", f"-fsanitize={sanitizer}", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "paper_2408_16551_amd", "csrc"), os.path.join(ROOT, "tests", "sched_driver.cpp"),
           "-o", str(exe), "-pthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "scenarios ok" in r.stdout


def test_next_request_of_a_stream_is_admitted_once_the_previous_is_issued():
    # R1's samples all go to step 1; R2 of the same stream is admitted at once
    # and takes step 2 while step 1 is still in flight; both complete in order.
    P, fps = 16, 4
    ops = [("add_stream", P, 0), ("submit", 0, P * 4), ("submit", 0, P * 4)]
    ops += [("admit", 0, 0), ("ready", 0, 1), ("step", 0, 0), ("admit", 0, 0), ("ready", 0, 2), ("step", 0, 0)]
    ev = sim(ops, max_active=1, frames_per_step=fps)
    assert [e["id"] for e in of(ev, "admit")] == [1, 2]
    assert step_items(ev) == [[(1, P * 4, 4)], [(2, P * 4, 4)]]
    assert not [e for e in of(ev, "complete") if e["id"]]
    ev = sim(ops + [("complete", 0, 0), ("complete", 0, 0)], max_active=1, frames_per_step=fps)
    assert [e["id"] for e in of(ev, "complete") if e["id"]] == [1, 2]


def test_a_request_still_issuing_holds_its_slot_and_stream():
    # R1 needs two steps: until its last samples are issued, R2 (same stream)
    # and R3 (another stream, no free slot) wait.
    P, fps = 16, 4
    ops = [("add_stream", P, 0), ("add_stream", P, 0), ("submit", 0, P * 8), ("submit", 0, P), ("submit", 1, P)]
    ops += [("admit", 0, 0), ("ready", 0, 1), ("step", 0, 0), ("admit", 0, 0)]
    ev = sim(ops, max_active=1, frames_per_step=fps)
    assert [e["id"] for e in of(ev, "admit")] == [1]
    ev = sim(ops + [("step", 0, 0), ("admit", 0, 0)], max_active=1, frames_per_step=fps)
    assert [e["id"] for e in of(ev, "admit")] == [1, 2]


def test_failed_step_ends_the_later_requests_of_its_streams():
    P, fps = 16, 4
    ops = [("add_stream", P, 0), ("add_stream", P, 0), ("submit", 0, P * 4), ("submit", 0, P * 4), ("submit", 1, P * 4)]
    ops += [("admit", 0, 0), ("ready", 0, 1), ("ready", 0, 3), ("step", 0, 0)]        # step 1: R1 and R3
    ops += [("admit", 0, 0), ("ready", 0, 2), ("step", 0, 0)]                         # step 2: R2
    ops += [("complete", 4, 0), ("complete", 0, 0)]                                   # step 1 fails
    ev = sim(ops, max_active=2, frames_per_step=fps)
    done = {e["id"]: e["status"] for e in of(ev, "complete") if e["id"]}
    assert done == {1: 4, 3: 4, 2: 4}


def test_empty_request_completes_after_the_earlier_request_of_its_stream():
    P = 16
    ops = [("add_stream", P, 0), ("submit", 0, P * 4), ("submit", 0, 0)]
    ops += [("admit", 0, 0), ("ready", 0, 1), ("step", 0, 0), ("admit", 0, 0), ("ready", 0, 2), ("step", 0, 0)]
    ev = sim(ops, max_active=2, frames_per_step=4)
    assert not [e for e in of(ev, "complete") if e["id"]]
    ev = sim(ops + [("complete", 0, 0), ("step", 0, 0)], max_active=2, frames_per_step=4)
    assert [e["id"] for e in of(ev, "complete") if e["id"]] == [1, 2]
