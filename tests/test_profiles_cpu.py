"""The committed profiler summaries stay reproducible (no GPU): every command
they give runs committed files with options those files accept, each
summary names the source SHA-1 it was measured on, and the HBM-traffic
summaries are the ones bench.py's traffic tables were taken from."""

import glob
import os
import re
import shlex
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2509_15879_amd import profile_workload  # noqa: E402

PROFILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")))
PARSERS = {"bench.py": bench.arg_parser, "paper_2509_15879_amd/profile_workload.py": profile_workload.arg_parser}
SHA = re.compile(r"\b[0-9a-f]{40}\b")


def commands(text):
    """(script, argv) of every `python3 $R/<script> ...` in a summary, with
    continuation lines joined."""
    joined = text.replace("\\\n", " ")
    out = []
    for m in re.finditer(r"python3 \$R/(\S+)([^\n]*)", joined):
        tail = re.split(r"\s(?:>|&&|\|)", m.group(2))[0]
        out.append((m.group(1), shlex.split(tail)))
    return out


def test_there_are_summaries():
    assert len(PROFILES) >= 5


@pytest.mark.parametrize("path", PROFILES, ids=os.path.basename)
def test_commands_run_committed_files_with_accepted_options(path):
    cmds = commands(open(path).read())
    assert cmds, "a summary gives the command that made it"
    for script, argv in cmds:
        assert os.path.isfile(os.path.join(ROOT, script)), script
        assert script in PARSERS, f"no parser known for {script}"
        PARSERS[script]().parse_args(argv)   # exits (fails the test) on an unknown option


@pytest.mark.parametrize("path", PROFILES, ids=os.path.basename)
def test_each_summary_names_its_source_sha(path):
    assert SHA.search(open(path).read()), "a summary names the kernel_source_sha1 it was measured on"


@pytest.mark.parametrize("key,summary", [("cfg3_fp64", "cycle_kernels_cfg3_1024x2048_hbm_traffic.txt"),
                                         ("cfg3_mixed", "cycle_kernels_cfg3_mixed_1024x2048_hbm_traffic.txt")])
def test_traffic_tables_come_from_their_summaries(key, summary):
    text = open(os.path.join(ROOT, "profiles", summary)).read()
    t = bench.TRAFFIC[key]
    assert t["sha1"] in SHA.findall(text)
    for fam, b in t["b_per_cell"].items():
        row = re.search(rf"^{fam}\s+\d+\s+[\d.]+\s+[\d.]+\s+[\d.]+\s+([\d.]+)", text, re.M)
        assert row and abs(float(row.group(1)) - b) < 0.01, fam
