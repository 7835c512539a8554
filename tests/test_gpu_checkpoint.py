"""Checkpoint and resume through the C ABI: a run saved between pulses and
resumed in a fresh context continues exactly as the uninterrupted run
(counter-based random numbers: same steps, same reactions, same counts)."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2509_03313_amd import workload as W  # noqa: E402


def say(*a):
    print("[gpu-test]", *a, flush=True)


@pytest.fixture(scope="module")
def g():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the device"
    from paper_2509_03313_amd import gsbs
    return gsbs


def _run_two(g, seed=77):
    wls = [W.multi_pulse(5 + i, n_pulses=3, dose_per_pulse=1.0, L=2000.0, avg_rate_gy_s=1e4, n_batches=2,
                         n_records=20) for i in range(2)]
    e = g.Engine([w.L for w in wls], seed, W.D_CONFIG, W.REACTIONS)
    for i, w in enumerate(wls):
        e.load_workload(w, inst=i)
    return e, wls


def test_resume_continues_exactly(g):
    e, wls = _run_two(g)
    t1 = 150e3  # ns: after the second pulse's batches, before the third pulse
    e.advance_to(t1)
    blob = e.save()
    say("checkpoint bytes", len(blob), "molecules", [e.n(i) for i in range(2)])
    t_end = max(w.t_end for w in wls)
    e.advance_to(t_end)
    ca = [e.counts(i) for i in range(2)]
    ga = [e.gvalues(i) for i in range(2)]
    na = [e.current_counts(i) for i in range(2)]
    sa = e.stats()
    e.close()
    f = g.Engine([w.L for w in wls], 12345, W.D_CONFIG, W.REACTIONS)
    f.load(blob, records=[w.records for w in wls])
    assert [f.time(i) for i in range(2)] == [t1, t1]
    f.advance_to(t_end)
    for i in range(2):
        assert np.array_equal(f.counts(i), ca[i]), i
        assert np.array_equal(f.gvalues(i), ga[i]), i
        assert np.array_equal(f.current_counts(i), na[i]), i
    assert f.stats()["reactions"] == sa["reactions"]
    f.close()


def test_checkpoint_keeps_chemistry_and_rejects_bad_input(g):
    e = g.Engine([1000.0, 1000.0], 3, W.D_CONFIG_O2, W.REACTIONS_O2)
    g.gsbs_set_first_order(e.ctx, W.FIRST_ORDER_O2)
    g.gsbs_set_sources(e.ctx, W.SOURCES_PH7)
    rng = np.random.default_rng(1)
    e.inject(0, 0.0, rng.uniform(-400, 400, size=(500, 3)).astype(np.float32),
             rng.integers(0, 8, size=500).astype(np.uint8))
    e.advance_to(5.0)
    blob = e.save()
    c0 = 10.0 ** rng.uniform(-8, -6, size=(4, 8))
    ref, _ = g.gsbs_numodes(e.ctx, c0, [1e3, 1e5, 1e7, 1e9])
    e.close()
    f = g.Engine([1000.0, 1000.0], 9, W.D_CONFIG, W.REACTIONS)  # other chemistry: replaced by the load
    f.load(blob)
    got, _ = g.gsbs_numodes(f.ctx, c0, [1e3, 1e5, 1e7, 1e9])
    assert np.array_equal(got, ref)
    assert f.n(0) > 0 and f.time(0) == 5.0
    f.close()
    with pytest.raises(g.GsbsError):  # another number of instances
        h = g.Engine(1000.0, 3, W.D_CONFIG, W.REACTIONS)
        try:
            h.load(blob)
        finally:
            h.close()
    with pytest.raises(g.GsbsError):  # other edges
        h = g.Engine([1000.0, 1500.0], 3, W.D_CONFIG, W.REACTIONS)
        try:
            h.load(blob)
        finally:
            h.close()
    h = g.Engine([1000.0, 1000.0], 3, W.D_CONFIG, W.REACTIONS)
    for bad in (blob[: len(blob) // 2], b"\x00" * 64, blob + b"\x01"):
        with pytest.raises(g.GsbsError):
            h.load(bad)
    h.close()


def test_corrupt_checkpoints_are_rejected_and_leave_the_context_intact(g):
    """A checkpoint whose molecule records or queued molecules are out of range
    (species byte, instance field, position, counts that differ from the
    molecules) fails with EINVAL before the context is touched: the context
    still runs as before."""
    L = 1000.0
    rng = np.random.default_rng(5)
    n = 300
    xyz = rng.uniform(-400, 400, size=(n, 3)).astype(np.float32)
    sp = rng.integers(0, 7, size=n).astype(np.uint8)
    e = g.Engine(L, 3, W.D_CONFIG, W.REACTIONS)
    g.gsbs_debug_set_state(e.ctx, xyz, sp, np.arange(n, dtype=np.uint64) + 1000, step=4, next_uid=5000)
    q_xyz = rng.uniform(-400, 400, size=(40, 3)).astype(np.float32)
    q_sp = rng.integers(0, 7, size=40).astype(np.uint8)
    e.inject(0, 10.0, q_xyz, q_sp, 100.0)
    e.set_records(0, [0.0, 5.0, 20.0])
    blob = e.save()
    e.close()
    rec = lambda k: xyz[k].tobytes() + np.int32(int(sp[k])).tobytes()  # noqa: E731
    at = blob.find(rec(7))
    assert at > 0 and blob.find(rec(7), at + 1) < 0
    q_at = blob.find(q_xyz.tobytes())
    assert q_at > 0

    def patch(off, data):
        return blob[:off] + data + blob[off + len(data):]

    meta = at + 12
    bad = {
        "species byte": patch(meta, bytes([40])),
        "instance field": patch(meta + 1, bytes([3])),
        "NaN position": patch(at, np.float32(np.nan).tobytes()),
        "position outside": patch(at, np.float32(L / 2).tobytes()),
        "counts differ": patch(meta, bytes([(int(sp[7]) + 1) % 7])),
        "queued species": patch(q_at + q_xyz.nbytes, bytes([9])),
        "queued position": patch(q_at, np.float32(-L).tobytes()),
    }
    h = g.Engine(L, 3, W.D_CONFIG, W.REACTIONS)
    h.load(blob, records=[[0.0, 5.0, 20.0]])
    h.advance_to(2.0)
    for name, b in bad.items():
        with pytest.raises(g.GsbsError) as ex:
            h.load(b)
        assert ex.value.code == -1, (name, str(ex.value))
    assert h.time(0) == 2.0  # still the state before the failed loads
    h.advance_to(20.0)
    got = h.counts(0)
    h.close()
    ref = g.Engine(L, 3, W.D_CONFIG, W.REACTIONS)
    ref.load(blob, records=[[0.0, 5.0, 20.0]])
    ref.advance_to(2.0)
    ref.advance_to(20.0)
    assert np.array_equal(got, ref.counts(0))
    ref.close()


_CHILD = r'''
import os, sys
import numpy as np
sys.path.insert(0, {root!r})
from paper_2509_03313_amd import gsbs, workload as W
mode, path, out = sys.argv[1], sys.argv[2], sys.argv[3]
wls = [W.multi_pulse(5 + i, n_pulses=3, dose_per_pulse=1.0, L=2000.0, avg_rate_gy_s=1e4, n_batches=2,
                     n_records=20) for i in range(2)]
e = gsbs.Engine([w.L for w in wls], 77, W.D_CONFIG, W.REACTIONS)
if mode == "resume":
    e.load(open(path, "rb").read(), records=[w.records for w in wls])
else:
    for i, w in enumerate(wls):
        e.load_workload(w, inst=i)
T = 100e3  # pulse period
t_end = max(w.t_end for w in wls)
if mode != "resume":
    for k in (1, 2):  # checkpoint at every pulse start after the first
        e.advance_to(k * T)
        open(path + ".tmp", "wb").write(e.save())
        os.replace(path + ".tmp", path)
        if mode == "crash" and k == 2:
            os._exit(3)  # the process dies after its last checkpoint
e.advance_to(t_end)
np.save(out, np.stack([e.counts(i) for i in range(2)]))
e.close()
'''


def test_resume_after_a_crash(tmp_path):
    """A run that dies after writing its checkpoint at the third pulse start is
    finished by a new process from that file; the records equal those of a
    run that checkpointed at the same times and never stopped."""
    import subprocess
    import torch
    assert torch.cuda.is_available(), "GPU tests need the device"
    root = os.path.dirname(HERE)
    script = tmp_path / "child.py"
    script.write_text(_CHILD.format(root=root))
    ck = str(tmp_path / "run.ckpt")

    def child(*args):
        return subprocess.run([sys.executable, str(script), *args], timeout=300).returncode

    assert child("full", str(tmp_path / "full.ckpt"), str(tmp_path / "full.npy")) == 0
    assert child("crash", ck, str(tmp_path / "never.npy")) == 3
    assert not (tmp_path / "never.npy").exists() and os.path.exists(ck)
    assert child("resume", ck, str(tmp_path / "resumed.npy")) == 0
    full = np.load(tmp_path / "full.npy")
    resumed = np.load(tmp_path / "resumed.npy")
    say("records", full.shape, "final counts", full[0, -1].tolist())
    assert np.array_equal(full, resumed)
