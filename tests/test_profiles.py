"""The committed rocprofv3 summaries: short text, each with the full command
that produced it, and every command runs committed files with options that
bench.py accepts."""
import glob
import os
import shlex

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*")))


def commands(path):
    return [line.lstrip("#").strip() for line in open(path)
            if line.lstrip("#").strip().startswith("cd /tmp")]


def test_profiles_exist():
    names = {os.path.basename(p) for p in PROFILES}
    assert "kernels_url_10M.txt" in names and "pmc_k_scatter_url_10M.txt" in names


@pytest.mark.parametrize("path", PROFILES, ids=os.path.basename)
def test_profile_is_a_short_summary_with_its_command(path):
    assert path.endswith((".txt", ".md"))
    assert os.path.getsize(path) < 16 * 1024
    assert commands(path), "no command line"


@pytest.mark.parametrize("path", PROFILES, ids=os.path.basename)
def test_profile_commands_run_committed_files(path):
    import bench
    for cmd in commands(path):
        words = shlex.split(cmd)
        prog = words[words.index("--") + 1:]
        assert prog[0] == "python3"
        script = prog[1].replace("$REPO/", "")
        assert script == "bench.py" and os.path.exists(os.path.join(ROOT, script))
        bench.arg_parser().parse_args(prog[2:])
        tool = words[words.index("rocprofv3"):words.index("--")]
        assert "--pmc" not in tool or not ({"-s", "--sys-trace", "-r", "--runtime-trace"} & set(tool))
