"""The C-ABI library loads and exports every entry point the header
declares (no compute call: runs without a GPU)."""
import os
import re
import subprocess

from paper_1801_10233_amd import spinlat as sl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spinlat.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sl_[a-z_0-9]+)\s*\(", text)))


def test_header_matches_binding_list():
    assert declared() == sorted(sl.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = sl.lib()
    for name in declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", sl.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sl_[a-z_0-9]+)$", out, flags=re.M))
    assert set(declared()) <= exported


def test_last_error_without_handle_is_a_string():
    assert isinstance(sl.lib().sl_last_error(None), bytes)


def test_library_has_gfx950_code_object():
    # the offload bundle of a hipcc build names its target
    data = open(sl.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_product_package_does_not_reach_the_oracle():
    pkg = os.path.join(ROOT, "paper_1801_10233_amd")
    bad = re.compile(r"(import\s+oracle|from\s+oracle|liboracle|\borc_[a-z])")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not bad.search(src), f


def test_static_mlp_eval_allocates_nothing():
    # the no-allocation entry point and its helpers call no device allocator
    # and take the static array only through its resolved device address
    src = open(os.path.join(ROOT, "paper_1801_10233_amd", "csrc", "sl_mlp_api.hip")).read()
    start = src.index("// sl_mlp_eval without device allocation.")
    body = src[start:]
    for bad in ("hipMalloc", "hipFree", "hipHostMalloc", "std::vector", "new ", "malloc("):
        assert bad not in body, bad
    # `scratch` appears only in its definition and in hipGetSymbolAddress
    code = re.sub(r"//[^\n]*", "", body)
    code = re.sub(r'"[^"\n]*"', '""', code)
    assert re.findall(r"\bscratch\b(?!_)", code) == ["scratch", "scratch"]
    assert "HIP_SYMBOL(scratch)" in code
