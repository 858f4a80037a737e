"""CPU checks of bench.py's contract that need no GPU: more than one GPU is
refused with a message, the recorded HBM traffic is only reported while the
profiled kernel sources are unchanged, the percentile helper is the
nearest-rank one, the timed steps issue exactly the work the reported
value counts (with stand-ins for torch and the library), and the sections
after the timed step run in child processes of their own."""
import ctypes
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_recorded_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    # The committed summary matches the committed sources.
    assert isinstance(bench.recorded_traffic(), int)
    # A summary taken from other sources is not used.
    text = open(bench.TRAFFIC_FILE).read()
    stale = tmp_path / "stale.md"
    stale.write_text(text.replace(bench.kernel_source_hash(), "0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.recorded_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.recorded_traffic() is None


def test_percentile_is_nearest_rank():
    xs = [5.0, 1.0, 4.0, 2.0, 3.0]
    assert bench.pct(xs, 50) == 3.0
    assert bench.pct(xs, 100) == 5.0
    assert bench.pct(xs, 1) == 1.0
    assert bench.pct(list(range(1, 101)), 99) == 99
    assert bench.pct([1.0, 2.0, 3.0, 4.0], 50) == 2.0


class _Ev:
    def record(self, stream=None):
        pass

    def synchronize(self):
        pass

    def elapsed_time(self, other):
        return 1.0


class _Stream:
    def wait_event(self, ev):
        pass


class _FakeTorch:
    """Just enough of torch for Pipeline's bookkeeping (no device)."""
    class cuda:  # noqa: N801
        Stream = _Stream

        @staticmethod
        def Event(enable_timing=False):  # noqa: N802
            return _Ev()

        @staticmethod
        def synchronize():
            pass

    int64 = "int64"
    uint8 = "uint8"

    class _T:
        def __init__(self, *shape):
            self.shape = shape

        def numel(self):
            n = 1
            for x in self.shape:
                n *= x
            return n

        def fill_(self, v):
            return self

        def __getitem__(self, k):
            return self

    @classmethod
    def empty(cls, *shape, dtype=None, device=None):
        return cls._T(*(shape[0] if isinstance(shape[0], tuple) else shape))

    zeros = empty


class _FakeCtx:
    log = []

    def __init__(self, dev=0):
        pass

    def batch_outputs(self, specs):
        recs = (_FakeHg.hg_block_job * len(specs))()
        for i, (_, b, k) in enumerate(specs):
            recs[i].block_size, recs[i].digest = b, k
        return recs, [None] * len(specs), [None] * len(specs)

    def device_job_table(self, recs):
        return ("table", tuple((r.digest, r.block_size) for r in recs))

    def run_batch(self, table, n, which="both", stream=None, host_roots=False, **kw):
        jobs = table[1] if isinstance(table, tuple) else tuple((r.digest, r.block_size) for r in table)
        assert len(jobs) == n
        self.log.append((which, host_roots, jobs))

    def chunk(self, data, *a, out=None, **kw):
        self.log.append(("chunk",))
        return out

    def similarity(self, *a, **kw):
        self.log.append(("similarity",))

    def close(self):
        pass


class _FakeJob(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_uint64), ("digest", ctypes.c_int32)]


class _FakeHg:
    hg_block_job = _FakeJob
    Context = _FakeCtx


def test_timed_steps_issue_exactly_the_counted_work():
    # K steps issue K launches of each kind of segment work, K early and K
    # late host second levels and K chunkings -- one pass of each of the
    # seven primitives per step, nothing for steps that did not run.
    class Data:
        device = "cpu"

        def numel(self):
            return 1 << 30
    for steps, slots in [(20, 10), (7, 10), (13, 4)]:
        _FakeCtx.log = []
        pipe = bench.Pipeline(_FakeTorch, _FakeHg, Data(), None, slots)
        pipe.run(5, steps)
        pipe.close()
        log = _FakeCtx.log
        short = [e for e in log if e[0] == "leaves" and len(e[2]) == len(bench.SHORT)]
        long_ = [e for e in log if e[0] == "leaves" and len(e[2]) == len(bench.LONG)]
        roots = [e for e in log if e[0] == "roots"]
        assert len(short) == len(long_) == steps
        assert all(e[2] == tuple(bench.BLOCK_JOBS[j] for j in bench.SHORT) for e in short)
        assert all(e[2] == tuple(bench.BLOCK_JOBS[j] for j in bench.LONG) for e in long_)
        assert len(roots) == 2 * steps and all(e[1] for e in roots)
        covered = sorted(j for e in roots for j in e[2])
        assert covered == sorted(bench.BLOCK_JOBS * steps)
        assert sum(e[0] == "chunk" for e in log) == steps
        assert sum(e[0] == "similarity" for e in log) == steps


def test_sections_run_in_child_processes(monkeypatch):
    # Each measurement section after the timed step runs as `bench.py
    # --section NAME` in a child process with the serving parameters passed
    # on; its last JSON line is the result, and a failing child is an error.
    monkeypatch.setattr(sys, "argv", ["bench.py", "--serve-requests", "123", "--serve-slots", "5"])
    args = bench.parse()
    calls = []

    class Done:
        def __init__(self, rc, out):
            self.returncode, self.stdout = rc, out

    def fake_run(cmd, **kw):
        calls.append(cmd)
        return Done(0, '[bench] noise\n{"section": "serving", "result": {"peak_GBps": 1.5}}\n')

    monkeypatch.setattr(subprocess, "run", fake_run)
    assert bench.run_section("serving", args) == {"peak_GBps": 1.5}
    cmd = calls[0]
    assert cmd[0] == sys.executable and cmd[1].endswith("bench.py")
    assert cmd[cmd.index("--section") + 1] == "serving"
    assert cmd[cmd.index("--serve-requests") + 1] == "123" and cmd[cmd.index("--serve-slots") + 1] == "5"
    monkeypatch.setattr(subprocess, "run", lambda cmd, **kw: Done(1, ""))
    try:
        bench.run_section("batched", args)
    except RuntimeError as e:
        assert "batched" in str(e)
    else:
        raise AssertionError("a failing section was not reported")


def test_default_run_composes_the_children(monkeypatch, capsys):
    # The default run: the step and each section from its child process,
    # one JSON line with the step's latency and ALU figures last.
    monkeypatch.setattr(sys, "argv", ["bench.py", "--no-cpu-baseline", "--no-sweep"])
    seen = []

    def fake_section(name, args):
        seen.append(name)
        if name == "step":
            return {"metric": "m", "value": 1.0, "step_alu": {"frac": 0.5}, "latency_ms": {"step_p50": 2.0}}
        return {"from": name}

    monkeypatch.setattr(bench, "run_section", fake_section)
    bench.main()
    out = capsys.readouterr().out.strip().splitlines()
    import json
    line = json.loads(out[-1])
    assert seen == ["step", "breakdown", "batched", "dedup", "serving"]
    assert line["breakdown"] == {"from": "breakdown"} and line["serving"] == {"from": "serving"}
    assert "similarity_sweep" not in line and "cpu_baseline" not in line
    assert list(line)[-2:] == ["step_alu", "latency_ms"]
