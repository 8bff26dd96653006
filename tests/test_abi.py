"""CPU checks of the C ABI: the library loads, exports every function that
include/jatam.h declares, and rejects bad arguments before any launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(jatam_\w+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2205_15311_amd import jatam
    if not os.path.exists(jatam.LIB_PATH):
        pytest.fail("libjatam.so is not built (run __graft_entry__.build())")
    return jatam.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "jatam_classify" in names and "jatam_classify_range" in names
    for name in names:
        assert hasattr(lib, name), name


def test_abi_version_and_strerror(lib):
    from paper_2205_15311_amd import jatam
    assert jatam.abi_version() >= 1
    for code in (0, -1, -2, -3, -99):
        assert isinstance(jatam.strerror(code), str)


@pytest.mark.parametrize("t,c,grid,runs", [(0, 8, 16, 20), (5, 8, 16, 20), (2, 3, 16, 20),
                                           (2, 8, 15, 20), (2, 8, 6, 20), (2, 8, 66, 20),
                                           (2, 8, 16, 0), (2, 8, 16, 65), (4, 32, 16, 1)])
def test_invalid_arguments_rejected(lib, t, c, grid, runs):
    out = ctypes.create_string_buffer(16)
    g = ctypes.c_uint64(0)
    assert lib.jatam_classify(ctypes.addressof(g), 1, t, c, grid, runs, 1, out, None) == -1
    assert lib.jatam_classify_range(0, 1, t, c, grid, runs, 1, out, None) == -1


def test_unsupported_grid(lib):
    out = ctypes.create_string_buffer(16)
    assert lib.jatam_classify_range(0, 1, 2, 8, 64, 20, 1, out, None) == -2


def test_range_beyond_space_rejected(lib):
    out = ctypes.create_string_buffer(16)
    assert lib.jatam_classify_range((1 << 24) - 1, 2, 2, 8, 16, 20, 1, out, None) == -1
    assert lib.jatam_classify_range(0, -1, 2, 8, 16, 20, 1, out, None) == -1
    # null buffers with n > 0
    assert lib.jatam_classify_range(0, 1, 2, 8, 16, 20, 1, None, None) == -1
    assert lib.jatam_classify(None, 1, 2, 8, 16, 20, 1, out, None) == -1


def test_empty_call_launches_nothing(lib):
    assert lib.jatam_classify(None, 0, 2, 8, 16, 20, 1, None, None) == 0
    assert lib.jatam_classify_range(0, 0, 2, 8, 16, 20, 1, None, None) == 0


@pytest.mark.parametrize("n,capacity", [(-1, 1024), (1, 0), (1, 100), (1, 32), (1, 1 << 25)])
def test_shape_histogram_rejects_bad_arguments(lib, n, capacity):
    recs = ctypes.create_string_buffer(16)
    table = ctypes.create_string_buffer(16 * 64)
    assert lib.jatam_shape_histogram(recs, n, table, capacity, None, None) == -1


def struct_fields(name):
    text = open(os.path.join(ROOT, "include", "jatam.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    m = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", text)
    assert m, name
    return re.findall(r"\b(\w+)\s*;", m.group(1))


def test_tuning_struct_matches_the_header():
    """The binding's jatam_tuning_t mirror has the header's fields, in order,
    all int."""
    import ctypes as ct
    from paper_2205_15311_amd import jatam
    assert [f for f, _ in jatam.Tuning._fields_] == struct_fields("jatam_tuning_t")
    assert all(t is ct.c_int for _, t in jatam.Tuning._fields_)
    assert ct.sizeof(jatam.Tuning) == 4 * len(jatam.Tuning._fields_)


def test_classify_batch_rejects_bad_arguments(lib):
    """jatam_classify_batch validates before touching the workspace."""
    out = ctypes.create_string_buffer(16)
    item = ctypes.create_string_buffer(24)
    # no workspace, bad colour count, bad run count
    assert lib.jatam_classify_batch(None, item, 1, 8, 20, 1, None, None, out, None, None) == -1
    assert lib.jatam_classify_batch(None, item, 1, 3, 20, 1, None, None, out, None, None) == -1
    assert lib.jatam_classify_batch(None, item, 1, 8, 0, 1, None, None, out, None, None) == -1


def test_ga_step_rejects_missing_workspaces(lib):
    from paper_2205_15311_amd import jatam
    p = jatam.GAParams()
    buf = ctypes.create_string_buffer(64)
    scr = jatam.ScreenStruct(None, None, 4, 0)
    # plain and screened generations without a batch workspace
    assert lib.jatam_ga_step(None, buf, buf, 4, 3, 8, 32, 20, 1, ctypes.byref(p), 0, None,
                             buf, buf, None) == -1
    assert lib.jatam_ga_step(None, buf, buf, 4, 3, 8, 32, 20, 1, ctypes.byref(p), 0,
                             ctypes.byref(scr), buf, buf, None) == -1


def test_screen_struct_matches_the_header():
    import ctypes as ct
    from paper_2205_15311_amd import jatam
    assert [f for f, _ in jatam.ScreenStruct._fields_] == struct_fields("jatam_screen_t")
    assert ct.sizeof(jatam.ScreenStruct) == 24


def test_true_class_rejects_bad_arguments(lib):
    """The true-class calls validate before touching a workspace."""
    out = ctypes.create_string_buffer(16)
    g = ctypes.c_uint64(0)
    h = ctypes.c_void_p()
    # no workspace; bad create arguments
    assert lib.jatam_true_class(None, ctypes.addressof(g), 1, 2, 8, 16, 100, out, None) == -1
    assert lib.jatam_true_class_range(None, 0, 1, 2, 8, 16, 100, out, None) == -1
    assert lib.jatam_truth_create(0, 16, 1, ctypes.byref(h)) == -1
    assert lib.jatam_truth_create(16, 0, 1, ctypes.byref(h)) == -1
    assert lib.jatam_truth_create(16, (1 << 18) + 1, 1, ctypes.byref(h)) == -1
    assert lib.jatam_truth_create(16, 16, 0, ctypes.byref(h)) == -1
    assert lib.jatam_truth_create(16, 16, 1, None) == -1
    assert lib.jatam_truth_destroy(None) == 0


def test_mlp_predict_rejects_bad_arguments(lib):
    """jatam_mlp_predict validates before touching a network."""
    buf = ctypes.create_string_buffer(64)
    for kind in (0, 1, 2, 3, -1):
        assert lib.jatam_mlp_predict(None, kind, buf, None, 2, 1, buf, None) == -1
    assert lib.jatam_mlp_score(None, buf, None, 2, 1, buf, None) == -1


def test_neighbourhood_rejects_bad_arguments(lib):
    buf = ctypes.create_string_buffer(64)
    # bad t or c; a range beyond the space; a space too large to gather from
    assert lib.jatam_single_mutants(None, 0, 1, 0, 8, buf, None) == -1
    assert lib.jatam_single_mutants(None, 0, 1, 2, 3, buf, None) == -1
    assert lib.jatam_single_mutants(None, (1 << 24) - 1, 2, 2, 8, buf, None) == -1
    assert lib.jatam_single_mutants(None, 0, 1, 2, 8, None, None) == -1
    assert lib.jatam_neighbourhood(buf, None, 1, 2, 8, buf, None) == -1
    assert lib.jatam_neighbourhood_space(buf, 0, 1, 3, 8, buf, None) == -1
    assert lib.jatam_neighbourhood_space(buf, (1 << 24) - 1, 2, 2, 8, buf, None) == -1
    # empty calls launch nothing
    assert lib.jatam_single_mutants(None, 0, 0, 2, 8, None, None) == 0
    assert lib.jatam_neighbourhood(None, None, 0, 2, 8, None, None) == 0
    assert lib.jatam_neighbourhood_space(None, 0, 0, 2, 8, None, None) == 0


def test_roulette_rejects_bad_arguments(lib):
    from paper_2205_15311_amd import jatam
    buf = ctypes.create_string_buffer(64)
    good = jatam.RouletteParams(5, 32, 1, 0.5)
    lam = (ctypes.c_double * 2)(0.5, 1.0)
    for bad in (jatam.RouletteParams(5, 0, 1, 0.5), jatam.RouletteParams(5, 65, 1, 0.5),
                jatam.RouletteParams(5, 32, 2, 0.5), jatam.RouletteParams(5, 32, 1, -1.0),
                jatam.RouletteParams(5, 32, 1, 65.0)):
        assert lib.jatam_roulette_offspring(buf, buf, 4, ctypes.byref(bad), 0, 4, buf, buf,
                                            None) == -1
        assert lib.jatam_fujiyama(ctypes.byref(bad), lam, 2, 1, 64, 10, 100, buf, buf, None,
                                  None) == -1
    # population size, missing buffers, rate and population limits, target
    assert lib.jatam_roulette_offspring(buf, buf, 0, ctypes.byref(good), 0, 4, buf, buf,
                                        None) == -1
    assert lib.jatam_roulette_offspring(buf, buf, 65537, ctypes.byref(good), 0, 4, buf, buf,
                                        None) == -1
    assert lib.jatam_roulette_offspring(buf, buf, 4, ctypes.byref(good), 0, 4, None, buf,
                                        None) == -1
    lam9 = (ctypes.c_double * 9)(*([0.5] * 9))
    assert lib.jatam_fujiyama(ctypes.byref(good), lam9, 9, 1, 64, 10, 100, buf, buf, None,
                              None) == -1
    assert lib.jatam_fujiyama(ctypes.byref(good), lam, 2, 1, 1025, 10, 100, buf, buf, None,
                              None) == -1
    assert lib.jatam_fujiyama(ctypes.byref(good), lam, 2, 1, 64, 33, 100, buf, buf, None,
                              None) == -1


def test_classify_variant_rejects_bad_arguments(lib):
    out = ctypes.create_string_buffer(64)
    assert lib.jatam_classify_variant(None, 0, 1, 2, 8, 16, 20, 1, 4, out, None) == -1
    assert lib.jatam_classify_variant(None, 0, 1, 0, 8, 16, 20, 1, 1, out, None) == -1
    assert lib.jatam_classify_variant(None, (1 << 24) - 1, 2, 2, 8, 16, 20, 1, 1, out, None) == -1
    assert lib.jatam_classify_variant(None, 0, 0, 2, 8, 16, 20, 1, 3, None, None) == 0


def test_autotune_cached_rejects_bad_arguments(lib):
    buf = ctypes.create_string_buffer(64)
    assert lib.jatam_batch_autotune_cached(None, b"/tmp/x", 0, 1, 2, 8, 16, 20, 1, buf, None,
                                           None, None) == -1
    assert "file" in __import__("paper_2205_15311_amd").strerror(-5)
