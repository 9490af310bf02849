"""The server's scheduling core (admission, FIFO, budget, watchdog, arena)
compiled with g++ against a fake executor and run on the CPU, plain and
under AddressSanitizer + UndefinedBehaviorSanitizer."""
import os
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "sched_test.cpp")


@pytest.mark.parametrize("flags", [["-O2"], ["-O1", "-g", "-fsanitize=address,undefined",
                                             "-fno-omit-frame-pointer"]],
                         ids=["plain", "asan_ubsan"])
def test_scheduler_native(flags):
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "sched_test")
        subprocess.check_call(["g++", "-std=c++17", "-Wall", "-pthread"] + flags + [SRC, "-o", exe])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "sched ok" in r.stdout
