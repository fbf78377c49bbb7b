"""Accuracy of the library's float64 sine and cosine (csrc/trig.hpp, used by
the U(1) row kernel): the header built for the host with g++ and compared with
glibc's sin and cos over random arguments in six ranges (including the
library fallback beyond 2^20) and over special arguments (signed zeros,
subnormals, multiples of pi/2 and their neighbours, quarter-period points).
Bound: 2 ulp of the reference result (measured: 1)."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2102_01031_amd", "csrc")


def test_trig_within_two_ulp(tmp_path):
    exe = tmp_path / "trig_acc"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC, "-o", str(exe),
                    os.path.join(HERE, "trig_accuracy.cpp")], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    rows = {}
    for line in out:
        parts = line.split()
        if len(parts) == 4:
            rows[parts[0]] = [float(v) for v in parts[1:]]
        elif len(parts) == 3 and parts[0] == "nan":
            assert parts[1] == "1" and parts[2] == "1"
    assert set(rows) == {"tiny", "quarter", "small", "medium", "large", "fallback", "special"}
    for name, errs in rows.items():
        assert max(errs) <= 2.0, (name, errs)
