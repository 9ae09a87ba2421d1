"""On-disk index file: the durable form of a multi-index (cell-contiguous storage).

Layout, little-endian:

  header (64 bytes)
    char[8] magic   "FBPQIDX1"
    u32 version     1
    u32 D, T, M, Kc
    u32 nsect       6 to 9
    u64 N
    u8[24] reserved (zero)
  nsect section records (32 bytes each)
    u32 kind        1=C1 2=C2 3=R 4=offsets 5=codes 6=ids (required, once each);
                    7=QL 8=SL (local codebooks, both or neither) 9=Rot (OPQ), optional
    u32 crc32       CRC-32 (IEEE 802.3, as zlib) of the section bytes
    u64 offset      byte offset of the section from the file start (64-aligned)
    u64 bytes       section size
    u64 reserved
  section payloads
    C1 f32 [T][D/2], C2 f32 [T][D/2], R f32 [M][Kc][D/M],
    offsets i64 [T*T+1], codes u8 [N][M] (storage order), ids u32 [N],
    QL, SL f32 [T][M/2][Kc][D/M], Rot f32 [D][D]
"""

from __future__ import annotations

import struct
import zlib

import numpy as np

from .gen import Index

MAGIC = b"FBPQIDX1"
VERSION = 1
HDR = struct.Struct("<8s5IIQ24s")
SEC = struct.Struct("<IIQQQ")
KINDS = ("C1", "C2", "R", "offsets", "codes", "ids", "QL", "SL", "Rot")


def _align(x: int, a: int = 64) -> int:
    return (x + a - 1) // a * a


def write_index(path: str, ix: Index) -> None:
    ix.check()
    arrays = [np.ascontiguousarray(ix.C1), np.ascontiguousarray(ix.C2), np.ascontiguousarray(ix.R),
              np.ascontiguousarray(ix.offsets), np.ascontiguousarray(ix.codes),
              np.ascontiguousarray(ix.ids)]
    kinds = [1, 2, 3, 4, 5, 6]
    for kind, a in ((7, ix.QL), (8, ix.SL), (9, ix.Rot)):
        if a is not None:
            arrays.append(np.ascontiguousarray(a))
            kinds.append(kind)
    pos = _align(HDR.size + SEC.size * len(arrays))
    recs = []
    for kind, a in zip(kinds, arrays):
        b = a.nbytes
        crc = zlib.crc32(memoryview(a).cast("B")) & 0xFFFFFFFF
        recs.append((kind, crc, pos, b, 0))
        pos = _align(pos + b)
    with open(path, "wb") as f:
        f.write(HDR.pack(MAGIC, VERSION, ix.D, ix.T, ix.M, ix.Kc, len(arrays), ix.N, b"\0" * 24))
        for r in recs:
            f.write(SEC.pack(*r))
        for r, a in zip(recs, arrays):
            f.seek(r[2])
            a.tofile(f)


def read_index(path: str) -> Index:
    with open(path, "rb") as f:
        magic, ver, D, T, M, Kc, nsect, N, _ = HDR.unpack(f.read(HDR.size))
        if magic != MAGIC or ver != VERSION or not 6 <= nsect <= 9:
            raise ValueError("not an FBPQ index file")
        recs = [SEC.unpack(f.read(SEC.size)) for _ in range(nsect)]
        shapes = {1: ((T, D // 2), np.float32), 2: ((T, D // 2), np.float32),
                  3: ((M, Kc, D // M), np.float32), 4: ((T * T + 1,), np.int64),
                  5: ((N, M), np.uint8), 6: ((N,), np.uint32),
                  7: ((T, M // 2, Kc, D // M), np.float32), 8: ((T, M // 2, Kc, D // M), np.float32),
                  9: ((D, D), np.float32)}
        out = {}
        for kind, crc, off, nbytes, _ in recs:
            if kind not in shapes or kind in out:
                raise ValueError(f"bad or repeated section kind {kind}")
            shape, dt = shapes[kind]
            f.seek(off)
            a = np.fromfile(f, dtype=dt, count=int(np.prod(shape))).reshape(shape)
            if a.nbytes != nbytes or (zlib.crc32(memoryview(a).cast("B")) & 0xFFFFFFFF) != crc:
                raise ValueError(f"section {KINDS[kind - 1]} corrupt")
            out[kind] = a
    ix = Index(D=D, T=T, M=M, Kc=Kc, C1=out[1], C2=out[2], R=out[3], offsets=out[4],
               codes=out[5], ids=out[6], QL=out.get(7), SL=out.get(8), Rot=out.get(9))
    ix.check()
    return ix
