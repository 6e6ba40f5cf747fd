"""Host-side contract of bench.py that needs no GPU: one GPU only, the
workload switch, and the source fingerprints that key the stored HBM traffic."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


@pytest.mark.parametrize("n", ["0", "2", "8"])
def test_more_than_one_gpu_is_refused(n):
    r = _run("--gpus", n)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_only_accepts_the_named_workloads():
    names = [name for name, _ in bench.EXTRA_PARTS]
    assert len(set(names)) == len(names)
    for want in ("decode", "recode", "sweep", "k_sweep", "single_generation"):
        assert want in names
    r = _run("--only", "no_such_workload")
    assert r.returncode == 2 and "invalid choice" in r.stderr


def test_source_hash_tracks_the_kernel_files(tmp_path, monkeypatch):
    """The fingerprint covers every listed source of a form, so editing any of
    them (or the order) changes it and the stored traffic no longer applies."""
    csrc = tmp_path / "paper_1909_02871_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in {f for files in bench.KERNEL_SOURCES.values() for f in files}:
        (csrc / f).write_bytes(b"source of " + f.encode())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h2, h1 = bench.kernel_source_hash(2), bench.kernel_source_hash(1)
    assert h2 != h1 and len(h2) == 64
    assert bench.kernel_source_hash(3) == h1   # forms 1 and 3 share their sources
    (csrc / "gf_types.h").write_bytes(b"changed")
    assert bench.kernel_source_hash(2) != h2 and bench.kernel_source_hash(1) != h1
    assert all(len(k[0]) == 64 and k[1] in bench.KERNEL_SOURCES for k in bench.MEASURED_TRAFFIC)


def _profile_bench_commands():
    """The bench.py command lines in the code blocks of the committed profile summaries."""
    import glob
    import re
    import shlex
    cmds = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        text = open(path).read().replace("\\\n", " ")
        blocks = re.findall(r"```\n(.*?)```", text, flags=re.S)
        for line in "\n".join(blocks).splitlines():
            line = line.strip()
            m = re.match(r'[A-Z][A-Z0-9_]*="python3 <repo>/bench\.py([^"]*)"', line)
            if m:
                cmds.append((os.path.basename(path), shlex.split(m.group(1))))
            elif "bench.py" in line:
                tail = line.split("bench.py", 1)[1]
                cmds.append((os.path.basename(path), [t for t in shlex.split(tail) if not t.startswith("$")]))
    return cmds


def test_profile_commands_run_committed_options():
    """Every bench.py command that a profile summary gives parses with the
    committed bench.py (its flags and workload names exist)."""
    cmds = _profile_bench_commands()
    assert len(cmds) >= 6
    parser = bench.make_parser()
    for where, args in cmds:
        try:
            parser.parse_args(args)
        except SystemExit:
            pytest.fail("%s: bench.py %s does not parse" % (where, " ".join(args)))
