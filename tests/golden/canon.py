"""Canonical byte form of factor entries for digest comparisons (no method
arithmetic: sign byte, 4-byte length, little-endian magnitude)."""
import hashlib


def canon_bytes(vals):
    out = bytearray()
    for v in vals:
        m = -v if v < 0 else v
        b = m.to_bytes((m.bit_length() + 7) // 8, "little")
        out += bytes([1 if v < 0 else 0]) + len(b).to_bytes(4, "little") + b
    return bytes(out)


def column_digest(C_col, L_col):
    h = hashlib.sha256()
    h.update(canon_bytes(C_col))
    h.update(b"|")
    h.update(canon_bytes(L_col))
    return h.hexdigest()
