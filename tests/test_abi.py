"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/fbpq.h, and validates index files without a GPU."""

import json
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fb():
    lib = os.path.join(ROOT, "paper_1404_1831_amd", "libfbpq.so")
    if not os.path.exists(lib):
        from paper_1404_1831_amd.build import build
        build()
    from paper_1404_1831_amd import fbpq
    return fbpq


def test_exports_match_header(fb):
    hdr = open(os.path.join(ROOT, "include", "fbpq.h")).read()
    declared = set(re.findall(r"\b(fbpq_[a-z_0-9]+)\s*\(", hdr))
    assert declared == set(fb.EXPORTS)
    for name in declared:
        assert hasattr(fb.lib, name)


def test_table_bytes_golden(fb):
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "table_memory.json")))
    tb, nb = fb.fbpq_table_bytes(g["T"], g["M"], g["K"])
    assert tb == g["dot_product_bytes"]
    assert nb < g["norm_bytes_below"]
    assert nb == (2 * g["T"] + g["M"] * g["K"]) * 4


def _write(tmp_path, ix, name="ix.bin"):
    p = str(tmp_path / name)
    synth.write_index(p, ix)
    return p


def test_index_file_roundtrip_and_check(fb, tmp_path):
    ix = synth.random_index(N=500, T=8, M=4, D=16, seed=1)
    p = _write(tmp_path, ix)
    info = fb.fbpq_index_file_check(p)
    assert (info.D, info.T, info.M, info.Kc, info.N) == (16, 8, 4, 256, 500)
    back = synth.read_index(p)
    for a in ("C1", "C2", "R", "offsets", "codes", "ids"):
        assert np.array_equal(getattr(back, a), getattr(ix, a))


def test_index_file_errors(fb, tmp_path):
    ix = synth.random_index(N=300, T=4, M=2, D=8, seed=2)
    p = _write(tmp_path, ix)
    raw = bytearray(open(p, "rb").read())
    with pytest.raises(fb.FbpqError) as e:
        fb.fbpq_index_file_check(str(tmp_path / "missing.bin"))
    assert e.value.code == fb.FBPQ_E_IO
    bad = bytearray(raw)
    bad[0:8] = b"NOTFBPQ!"
    (tmp_path / "magic.bin").write_bytes(bytes(bad))
    with pytest.raises(fb.FbpqError) as e:
        fb.fbpq_index_file_check(str(tmp_path / "magic.bin"))
    assert e.value.code == fb.FBPQ_E_FORMAT
    bad = bytearray(raw)
    bad[-5] ^= 0xFF  # payload byte of the ids section: CRC must catch it
    (tmp_path / "crc.bin").write_bytes(bytes(bad))
    with pytest.raises(fb.FbpqError) as e:
        fb.fbpq_index_file_check(str(tmp_path / "crc.bin"))
    assert e.value.code == fb.FBPQ_E_FORMAT
    (tmp_path / "short.bin").write_bytes(bytes(raw[:len(raw) // 2]))
    with pytest.raises(fb.FbpqError) as e:
        fb.fbpq_index_file_check(str(tmp_path / "short.bin"))
    assert e.value.code == fb.FBPQ_E_FORMAT
    # decreasing offsets with valid CRCs
    ix2 = synth.random_index(N=300, T=4, M=2, D=8, seed=2)
    ix2.offsets = ix2.offsets.copy()
    ix2.offsets[3], ix2.offsets[4] = ix2.offsets[4] + 1, ix2.offsets[3]
    p2 = str(tmp_path / "offs.bin")
    import zlib
    # write bypassing Index.check so the bad offsets reach the file
    arrays = [ix2.C1, ix2.C2, ix2.R, ix2.offsets, ix2.codes, ix2.ids]
    from synth.indexfile import HDR, SEC, MAGIC, _align
    pos = _align(HDR.size + SEC.size * 6)
    recs = []
    for k, a in enumerate(arrays):
        a = np.ascontiguousarray(a)
        recs.append((k + 1, zlib.crc32(a.tobytes()) & 0xFFFFFFFF, pos, a.nbytes, 0))
        pos = _align(pos + a.nbytes)
    with open(p2, "wb") as f:
        f.write(HDR.pack(MAGIC, 1, ix2.D, ix2.T, ix2.M, ix2.Kc, 6, ix2.N, b"\0" * 24))
        for r in recs:
            f.write(SEC.pack(*r))
        for r, a in zip(recs, arrays):
            f.seek(r[2])
            np.ascontiguousarray(a).tofile(f)
    with pytest.raises(fb.FbpqError) as e:
        fb.fbpq_index_file_check(p2)
    assert e.value.code == fb.FBPQ_E_FORMAT
    assert "offsets" in str(e.value)


def _write_sections(path, ix, sections):
    """A file with the given (kind, array) sections in that order, CRCs valid."""
    import zlib
    from synth.indexfile import HDR, SEC, MAGIC, _align
    pos = _align(HDR.size + SEC.size * len(sections))
    recs = []
    for kind, a in sections:
        a = np.ascontiguousarray(a)
        recs.append((kind, zlib.crc32(a.tobytes()) & 0xFFFFFFFF, pos, a.nbytes, 0))
        pos = _align(pos + a.nbytes)
    with open(path, "wb") as f:
        f.write(HDR.pack(MAGIC, 1, ix.D, ix.T, ix.M, ix.Kc, len(sections), ix.N, b"\0" * 24))
        for r in recs:
            f.write(SEC.pack(*r))
        for r, (_, a) in zip(recs, sections):
            f.seek(r[2])
            np.ascontiguousarray(a).tofile(f)


def test_index_file_optional_sections(fb, tmp_path):
    """Local codebooks (QL, SL) and the OPQ rotation travel in optional
    sections: written, read back and checked natively; QL without SL, a
    repeated kind and a corrupt optional section are format errors."""
    import dataclasses
    base = synth.random_index(N=400, T=8, M=4, D=16, seed=3)
    ix = dataclasses.replace(synth.with_local_codebooks(base, seed=4), Rot=synth.random_rotation(16, seed=6))
    p = _write(tmp_path, ix)
    info = fb.fbpq_index_file_check(p)
    assert (info.D, info.T, info.M, info.N) == (16, 8, 4, 400)
    back = synth.read_index(p)
    for a in ("C1", "C2", "R", "offsets", "codes", "ids", "QL", "SL", "Rot"):
        assert np.array_equal(getattr(back, a), getattr(ix, a)), a
    req = [(1, ix.C1), (2, ix.C2), (3, ix.R), (4, ix.offsets), (5, ix.codes), (6, ix.ids)]
    cases = {"ql_only.bin": req + [(7, ix.QL)],
             "twice.bin": req + [(9, ix.Rot), (9, ix.Rot)],
             "missing.bin": req[:5] + [(9, ix.Rot)],
             "rot_shape.bin": req + [(9, ix.Rot[:8])]}
    for name, secs in cases.items():
        _write_sections(str(tmp_path / name), ix, secs)
        with pytest.raises(fb.FbpqError) as e:
            fb.fbpq_index_file_check(str(tmp_path / name))
        assert e.value.code == fb.FBPQ_E_FORMAT, name
    raw = bytearray(open(p, "rb").read())
    raw[-3] ^= 0x40  # a payload byte of the rotation, the last section
    (tmp_path / "rot_crc.bin").write_bytes(bytes(raw))
    with pytest.raises(fb.FbpqError) as e:
        fb.fbpq_index_file_check(str(tmp_path / "rot_crc.bin"))
    assert e.value.code == fb.FBPQ_E_FORMAT


def test_invalid_arguments_without_gpu(fb):
    with pytest.raises(fb.FbpqError) as e:
        fb.fbpq_table_bytes(0, 8, 256)
    assert e.value.code == fb.FBPQ_E_INVALID
    with pytest.raises(fb.FbpqError) as e:
        fb.fbpq_set_option(None, "prefix", 4)
    assert e.value.code == fb.FBPQ_E_INVALID


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of fbpq_index_desc and fbpq_info_t have the C
    layout: a small C program built against include/fbpq.h prints sizeof and
    every field's offset, and the binding must agree field by field."""
    import ctypes
    import subprocess

    from paper_1404_1831_amd import fbpq as fbm

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = {"fbpq_index_desc": fbm.IndexDesc, "fbpq_info_t": fbm.Info}
    body = []
    for cname, py in structs.items():
        body.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            body.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "fbpq.h"\nint main(void) {\n'
                   + "\n".join(body) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (ln.split() for ln in out if ln)}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits at once with a message (one GPU only)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
