"""The oracle reproduces every hand-worked alignment in tests/golden."""
import pytest

import oracle
from golden_cases import load
from textbook import linear_sw
from workloads.gen import SeqSet

CASES = load()


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_golden_oracle(c):
    r = oracle.align_pairs(SeqSet.from_list([c["query"]]), SeqSet.from_list([c["target"]]),
                           c["S"], c["o"], c["e"], mode=c["mode"], ends=c["ends"] or None,
                           traceback=True, threads=1)
    got = (int(r["score"][0]), int(r["q_begin"][0]), int(r["q_end"][0]),
           int(r["t_begin"][0]), int(r["t_end"][0]), oracle.cigar_string(r["cigars"][0]))
    assert got == (c["score"], c["q_begin"], c["q_end"], c["t_begin"], c["t_end"], c["cigar"])


def test_textbook_example_linear_sw():
    c = [x for x in CASES if x["name"] == "sw_textbook"][0]
    assert linear_sw(c["query"], c["target"], c["S"], 2) == 13
