"""Host-side checks of the C ABI (no GPU needed, no kernel is launched).

* the library loads and exports every function declared in
  include/inplace_merge.h;
* argument validation returns the documented status codes before any device
  work (bad dtype, negative length, NULL pointer) and sets the thread-local
  message;
* the Python binding refuses host tensors instead of falling back to the CPU.
"""
import ctypes
import os
import re

import pytest

import paper_2005_12648_amd as im

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "inplace_merge.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_parses():
    names = declared_functions()
    for must in ("inplace_merge", "inplace_merge_kv", "batched_inplace_merge",
                 "batched_inplace_merge_kv", "inplace_merge_sort", "im_corank", "im_rotate",
                 "merge_model_train", "inplace_merge_learned", "inplace_merge_last_error"):
        assert must in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    lib = im.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def _err(lib):
    return lib.inplace_merge_last_error().decode()


def test_validation_codes_without_device_work():
    lib = im.load()
    vp = ctypes.c_void_p
    fake = vp(0x1000)   # never dereferenced: validation fails first
    assert lib.inplace_merge(fake, 4, 4, 9, None) == -2
    assert "dtype" in _err(lib)
    assert lib.inplace_merge(fake, -1, 4, 0, None) == -1
    assert "negative" in _err(lib)
    assert lib.inplace_merge(None, 4, 4, 0, None) == -1
    assert "null" in _err(lib)
    assert lib.inplace_merge_kv(fake, None, 3, 3, 0, 0, None) == -1
    assert lib.inplace_merge_kv(fake, fake, 3, 3, 0, 17, None) == -2
    assert lib.batched_inplace_merge(fake, None, 5, 0, None) == -1
    assert lib.batched_inplace_merge(fake, fake, -5, 0, None) == -1
    assert lib.batched_inplace_merge(fake, fake, 5, 9, None) == -2
    assert lib.batched_inplace_merge_kv(fake, None, fake, 5, 0, 0, None) == -1
    assert lib.batched_inplace_merge_sized(fake, None, 5, 100, 0, 0, None) == -1
    assert lib.batched_inplace_merge_sized(fake, fake, -5, 100, 0, 0, None) == -1
    assert lib.batched_inplace_merge_kv_sized(fake, fake, fake, 5, 100, 0, 0, 9, None) == -2
    assert lib.merge_model_train(None, fake, 4, 4, 0, None, None) == -1
    assert lib.inplace_merge_last_stats(None) == -1
    assert lib.inplace_merge_sort(fake, -3, 0, None) == -1
    assert lib.im_rotate(fake, 3, 4, 3, None) == -2
    assert lib.im_corank(fake, 3, 3, 0, None, 5, None, None, None) == -1
    # captured graph, leaf configuration and autotuner entry points
    out = vp()
    assert lib.batched_inplace_merge_graph(None, fake, fake, 4, 100, 0, 0, None) == -1
    assert lib.batched_inplace_merge_graph(ctypes.byref(out), fake, fake, 4, 100, 0, 9, None) == -2
    assert lib.batched_inplace_merge_graph(ctypes.byref(out), fake, fake, 0, 100, 0, 0, None) == -1
    assert lib.batched_inplace_merge_graph(ctypes.byref(out), None, fake, 4, 100, 0, 0, None) == -1
    assert out.value is None
    assert lib.im_graph_launch(None, None) == -1
    assert lib.im_graph_cooperative(None) == 0
    assert lib.im_graph_destroy(None) == 0
    assert lib.inplace_merge_set_config(4) == -1
    assert lib.inplace_merge_set_config(-2) == -1
    assert lib.inplace_merge_set_config(-1) == 0
    assert lib.inplace_merge_autotune(fake, fake, 4, 100, 0, 9, -1, 3, None, None, None) == -2
    assert lib.inplace_merge_autotune(fake, fake, 4, 100, 0, 0, 7, 3, None, None, None) == -2
    assert lib.inplace_merge_autotune(fake, fake, 4, 100, 0, 0, -1, 0, None, None, None) == -1
    assert lib.inplace_merge_autotune(None, fake, 4, 100, 0, 0, -1, 3, None, None, None) == -1
    # method variants and comparators
    assert lib.inplace_merge_variant(fake, 4, 4, 0, 2, 0, None) == -1
    assert lib.inplace_merge_variant(fake, 4, 4, 0, 0, 5, None) == -1
    assert lib.inplace_merge_variant(fake, 4, 4, 7, 0, 0, None) == -2
    assert lib.im_divide(fake, 4, 4, 0, 3, 2, fake, None) == -1
    assert lib.im_divide(fake, 4, 4, 0, 0, 25, fake, None) == -1
    assert lib.im_divide(fake, 4, 4, 0, 0, 2, None, None) == -1
    assert lib.im_rotate_cs(fake, 3, 4, 2, None) == -2
    assert lib.im_rotate_cs(fake, 0, 4, 4, None) == 0
    assert lib.merge_out_of_place(fake, fake, 4, 4, 0, None) == -1     # overlap
    assert lib.merge_out_of_place(fake, None, 4, 4, 0, None) == -1
    assert lib.inplace_merge_buffered(fake, -1, 4, 0, None) == -1
    assert lib.inplace_merge_buffered(fake, 0, 4, 0, None) == 0
    # empty work is a successful no-op that touches nothing
    assert lib.inplace_merge(None, 0, 0, 0, None) == 0
    assert lib.inplace_merge(fake, 0, 7, 0, None) == 0
    assert lib.im_rotate(fake, 0, 7, 4, None) == 0


def test_binding_rejects_host_tensors():
    import torch
    with pytest.raises(ValueError, match="HIP device"):
        im.inplace_merge(torch.arange(8, dtype=torch.int32), 4)
    with pytest.raises(ValueError):
        im.rotate(torch.arange(8, dtype=torch.int32), 4)


def test_no_oracle_in_product_path():
    # the product package never imports the test oracle
    pkg = os.path.join(ROOT, "paper_2005_12648_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt, f


def test_rows_validation_without_device_work():
    lib = im.load()
    fake = ctypes.c_void_p(0x1000)      # never dereferenced: validation fails first
    assert lib.inplace_merge_rows(fake, 4, 4, 64, 9, None) == -2            # dtype
    assert lib.inplace_merge_rows(fake, -1, 4, 64, 0, None) == -1
    assert lib.inplace_merge_rows(None, 4, 4, 64, 0, None) == -1
    assert lib.inplace_merge_rows(fake, 4, 4, 0, 0, None) == -1             # row bytes
    assert lib.inplace_merge_rows(fake, 4, 4, 6, 0, None) == -1             # not a multiple of 4
    assert lib.inplace_merge_rows(fake, 4, 4, 12, 2, None) == -1            # 8-byte key
    assert lib.inplace_merge_rows(fake, 4, 4, 81924, 0, None) == -1         # too wide
    assert "too large" in _err(lib)
    assert lib.inplace_merge_rows(fake, 4, 4, 81928, 0, None) == -1         # 8-byte chunks
    assert lib.inplace_merge_rows(ctypes.c_void_p(0x1002), 4, 4, 64, 0, None) == -1   # alignment
    assert lib.inplace_merge_rows(fake, 0, 9, 64, 0, None) == 0             # nothing to merge
    assert lib.inplace_merge_rows_workspace_bytes(-1, 64, 0) == 0
    assert lib.inplace_merge_rows_workspace_bytes(100, 0, 0) == 0


def _declaration(name):
    """Parameter list of a header declaration, whitespace-normalised."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"([A-Za-z_][A-Za-z0-9_ \*]*?)\b" + name + r"\s*\(([^)]*)\)\s*;", src)
    assert m, name
    ret = " ".join(m.group(1).split())
    args = [" ".join(a.replace("*", " * ").split()) for a in m.group(2).split(",")]
    # keep the types only (drop the parameter names)
    types = []
    for a in args:
        words = a.split(" ")
        if words == ["void"]:
            continue
        types.append(" ".join(words[:-1]) if len(words) > 1 and words[-1] != "*" else a)
    return ret, types


def test_boundary_matches_the_scope_table():
    # the calls of the boundary, with the argument types they are specified with
    want = {
        "inplace_merge": ("int", ["void *", "int64_t", "int64_t", "int", "hipStream_t"]),
        "inplace_merge_kv": ("int", ["void *", "void *", "int64_t", "int64_t", "int", "int",
                                     "hipStream_t"]),
        "batched_inplace_merge": ("int", ["void *", "const int64_t *", "int64_t", "int",
                                          "hipStream_t"]),
        "batched_inplace_merge_kv": ("int", ["void *", "void *", "const int64_t *", "int64_t",
                                             "int", "int", "hipStream_t"]),
        "inplace_merge_workspace_bytes": ("size_t", ["int64_t", "int"]),
        "inplace_merge_set_workspace": ("int", ["void *", "size_t"]),
        "inplace_merge_last_error": ("const char *", []),
        "merge_model_train": ("int", ["merge_model * *", "const void *", "int64_t", "int64_t",
                                      "int", "const merge_train_cfg *", "hipStream_t"]),
        "inplace_merge_learned": ("int", ["void *", "int64_t", "int64_t", "int",
                                          "const merge_model *", "hipStream_t"]),
        "merge_model_save": ("int", ["const merge_model *", "const char *"]),
        "merge_model_load": ("int", ["merge_model * *", "const char *"]),
        "merge_model_free": ("int", ["merge_model *"]),
        "inplace_merge_last_stats": ("int", ["merge_stats *"]),
    }
    for name, (ret, types) in want.items():
        got_ret, got_types = _declaration(name)
        assert got_ret.endswith(ret), (name, got_ret)
        assert got_types == types, (name, got_types)
