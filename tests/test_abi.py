"""Host-side checks of the C ABI: the library loads, exports every declared entry point, and
rejects invalid geometries before touching a device (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "fastfocus.h")


def _lib():
    from paper_2004_13904_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2004_13904_amd import build
        build.build(verbose=False)
    return L, L.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:ff_status|const char \*)\s*\**\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("build_spectra", "apply_G", "apply_GT", "apply_G_block", "gkb_project",
                     "rsvd_project", "irls_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L, lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(L.EXPORTS) == set(declared_functions())


def geom(L, **kw):
    s = dict(sx=8, sy=8, nz=2, dx=20.0, dy=20.0, z_edges=(0.0, 20.0, 40.0), kernel="gravity")
    s.update(kw)
    return L.make_geometry(s)


@pytest.mark.parametrize("kw,code", [
    (dict(z_edges=(1.0, 20.0, 40.0)), -1),            # station plane must be z = 0
    (dict(z_edges=(0.0, 20.0, 20.0)), -1),            # strictly increasing layers
    (dict(dx=-1.0), -1),
    (dict(sx=0), -2),
])
def test_invalid_geometry_is_rejected_on_the_host(kw, code):
    L, lib = _lib()
    g, keep = geom(L, **kw)
    h = C.c_void_p()
    rc = lib.build_spectra(C.byref(g), L.FF_F32, None, C.byref(h))
    assert rc == code
    assert lib.ff_last_error().decode()
    assert not h.value


def test_wraparound_embedding_is_rejected():
    L, lib = _lib()
    g, keep = geom(L)
    g.nfft_x = 8            # s_x + n_x - 1 = 15 > 8: circular wrap-around
    h = C.c_void_p()
    assert lib.build_spectra(C.byref(g), L.FF_F32, None, C.byref(h)) == -2
    g.nfft_x = 24           # not a power of two
    assert lib.build_spectra(C.byref(g), L.FF_F32, None, C.byref(h)) == -7


def test_bad_dtype_and_null_arguments():
    L, lib = _lib()
    g, keep = geom(L)
    h = C.c_void_p()
    assert lib.build_spectra(C.byref(g), 7, None, C.byref(h)) == -3
    assert lib.build_spectra(None, 0, None, C.byref(h)) == -1
    assert lib.apply_G(None, None, None, None, None, None) == -1
    assert lib.ff_free_spectra(None) == -1


def test_spectra_load_rejects_foreign_and_missing_files(tmp_path):
    # the magic and version are read before any device call
    L, lib = _lib()
    h = C.c_void_p(123)
    missing = str(tmp_path / "none.ffs").encode()
    assert lib.ff_spectra_load(missing, None, C.byref(h)) == L.FF_EINVAL and h.value is None
    junk = tmp_path / "junk.ffs"
    junk.write_bytes(b"NOTSPECTRA" + bytes(200))
    assert lib.ff_spectra_load(str(junk).encode(), None, C.byref(h)) == L.FF_EINVAL
    assert b"not a spectra file" in lib.ff_last_error()
    assert lib.ff_spectra_save(None, b"x") == L.FF_EINVAL


@pytest.mark.parametrize("n,dtype,inverse,count,code", [
    (12, 0, 0, 1, -2),        # not a power of two
    (4, 0, 0, 1, -2),         # below the smallest transform
    (4096, 1, 0, 1, -2),      # above the largest
    (64, 2, 0, 1, -3),        # unknown dtype
    (64, 0, 2, 1, -1),        # inverse must be 0 or 1
    (64, 0, 0, -1, -2),       # negative count
    (64, 0, 0, 0, 0),         # nothing to do
])
def test_fft_1d_rejects_bad_arguments_before_launching(n, dtype, inverse, count, code):
    L, lib = _lib()
    p = C.c_void_p(16)        # never dereferenced: validation precedes any device work
    assert lib.ff_fft_1d(n, dtype, inverse, 0, count, p, p, p, None) == code
    assert lib.ff_fft_1d(64, 0, 0, 0, 1, None, p, p, None) == -1
    for plan in (-1, 3):      # stage plans 0, 1 and 2 only
        assert lib.ff_fft_1d(64, 0, 0, plan, 1, p, p, p, None) == -1


@pytest.mark.parametrize("compiler,lang", [("gcc", "c"), ("g++", "c++")])
def test_header_compiles_as_plain_c_and_cpp(compiler, lang, tmp_path):
    """The boundary header is self-contained C (plain pointers, fixed-width integers, no torch or
    HIP types) and also valid C++."""
    import shutil
    import subprocess
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    r = subprocess.run([compiler, "-fsyntax-only", "-x", lang, "-Wall", "-Wextra", "-Werror", HEADER],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_every_entry_point_rejects_null_arguments():
    # NULL handles and buffers, zero sizes: every entry point returns FF_EINVAL with a message
    # naming itself, before any device call (so this runs without a GPU); freeing a NULL plan
    # is a no-op
    L, lib = _lib()
    for name in L.EXPORTS:
        if name in ("ff_last_error", "ff_multi_free"):
            continue
        fn = getattr(lib, name)
        args = []
        for t in fn.argtypes:
            if issubclass(t, (C._Pointer, C.c_void_p, C.c_char_p)):
                args.append(None)
            elif t in (C.c_double, C.c_float):
                args.append(0.0)
            else:
                args.append(0)
        assert fn(*args) == -1, name
        assert lib.ff_last_error().decode().startswith(name + ":"), name
    assert lib.ff_multi_free(None) == 0


def _header_struct_fields(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r";", text).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        names = decl.split(None, 1)[1] if not decl.startswith("const") else decl.split("*", 1)[1]
        fields += [v.strip().lstrip("*") for v in names.split(",")]
    return fields


@pytest.mark.parametrize("c_name,py_name", [("ff_tuning", "FFTuning"), ("ff_irls_params", "FFIrlsParams"),
                                            ("ff_geometry", "FFGeometry")])
def test_binding_structs_match_the_header(c_name, py_name):
    # the ctypes mirrors of the ABI structs list the header's fields in the header's order
    from paper_2004_13904_amd import _lib as L
    py = [f[0] for f in getattr(L, py_name)._fields_]
    hdr = _header_struct_fields(c_name)
    # Python cannot name a field "lambda"
    assert [("lam" if f == "lambda" else f) for f in hdr] == py
