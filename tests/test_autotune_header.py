"""The autotuner's header writer (CPU): the launch-shape header it writes compiles and
holds the chosen values, and the committed header's values are consistent."""
import os
import re
import shutil
import subprocess

import pytest

from paper_1406_4173_amd import autotune

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED = os.path.join(HERE, "..", "paper_1406_4173_amd", "csrc", "tuned.h")


def values(text):
    return {k: int(v) for k, v in re.findall(r"constexpr int64_t (tuned_\w+) = (\d+);", text)}


def test_written_header_holds_the_choice_and_compiles(tmp_path):
    out = tmp_path / "tuned.h"
    autotune.write_header(str(out), 2000, 5000, 256, 1, ["a sweep row", "chosen: ..."], (500, 1000, 200000))
    text = out.read_text()
    assert values(text) == {"tuned_small_range": 2000, "tuned_mid_range": 5000, "tuned_spg_div": 256,
                            "tuned_dense_shift": 1, "tuned_dsk_small_range": 500, "tuned_dsk_mid_range": 1000,
                            "tuned_dsk_group_work": 200000}
    assert "//   a sweep row" in text
    if shutil.which("g++") is None:
        pytest.skip("no host compiler")
    src = tmp_path / "use.cpp"
    src.write_text('#include "tuned.h"\nstatic_assert(bcpp::tuned_mid_range == 5000, "");\nint main() {}\n')
    subprocess.run(["g++", "-std=c++17", "-fsyntax-only", "-I", str(tmp_path), str(src)], check=True)


def test_committed_header_is_consistent():
    v = values(open(TUNED).read())
    assert set(v) == {"tuned_small_range", "tuned_mid_range", "tuned_spg_div", "tuned_dense_shift",
                      "tuned_dsk_small_range", "tuned_dsk_mid_range", "tuned_dsk_group_work"}
    assert 0 <= v["tuned_small_range"] <= v["tuned_mid_range"]
    assert 0 <= v["tuned_dsk_small_range"] <= v["tuned_dsk_mid_range"]
    assert v["tuned_dsk_group_work"] >= 0
    assert v["tuned_spg_div"] >= 1
    assert 0 <= v["tuned_dense_shift"] <= 63
