"""Host-side logic of bench.py (no GPU): the code text that decides whether
committed HBM-traffic counters still describe the kernels."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_code_text_ignores_comments_and_spacing(bench):
    a = "int f(int x)\n{\n    return x + 1;   // one more\n}\n"
    b = "/* the successor */\nint f(int x) {\n  return x + 1;\n}"
    assert bench.code_text(a) == bench.code_text(b) == "int f(int x) { return x + 1; }"


def test_code_text_sees_code_changes(bench):
    a = "int f(int x) { return x + 1; }"
    b = "int f(int x) { return x + 2; }"
    assert bench.code_text(a) != bench.code_text(b)
    # a comment marker inside a block comment, and one block comment spanning lines
    c = "int g; /* a // b\n c */ int h;"
    assert bench.code_text(c) == "int g; int h;"


def test_kernel_sources_digest_is_16_hex_digits(bench):
    d = bench.kernel_sources_digest()
    assert len(d) == 16 and int(d, 16) >= 0
