"""Host emulation of the 16-bit operand encodings of the mixed-precision
products (test side only): the exact values the MFMA instructions are fed,
so that a GPU product can be checked against an FP64 product of the same
operands within the FP32 accumulation error bound."""
import numpy as np

U32 = 2.0 ** -24   # unit roundoff of FP32 accumulation


def bf16(x):
    """Round FP32 values to bfloat16 (nearest, ties to even); float64 out."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def fp16(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


def split_bf16(x):
    """x (FP32) = hi + lo with hi = bf16(x), lo = bf16(x - hi)."""
    x32 = np.asarray(x, dtype=np.float32)
    hi = bf16(x32)
    lo = bf16((x32.astype(np.float64) - hi).astype(np.float32))
    return hi, lo


def untile(flat, R, K):
    """Decode a fragment-tiled 16-bit operand (R x K; 16 x 32 blocks of 512
    entries, block (rb, kb) at (rb * nkb + kb) * 512, lane t = 16 g + r holding
    X(16 rb + r, 32 kb + 8 g + e) at 8 t + e) into (X, padding)."""
    nrb, nkb = -(-R // 16), -(-K // 32)
    b = np.asarray(flat).reshape(nrb, nkb, 4, 16, 8)            # (rb, kb, g, r, e)
    full = b.transpose(0, 3, 1, 2, 4).reshape(nrb * 16, nkb * 32)
    pad = np.concatenate([full[R:, :].ravel(), full[:R, K:].ravel()])
    return full[:R, :K], pad


def bits16(x, kind, e=None):
    """uint16 patterns of the 16-bit encoding of the FP32 matrix x (hi, lo):
    bf16 / split bf16 round to nearest even, fp16 after the column scaling 2^-e_j."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    if kind == "fp16":
        y = (x.astype(np.float64) * np.exp2(-np.asarray(e, dtype=np.float64))[None, :]).astype(np.float32)
        return y.astype(np.float16).view(np.uint16), None
    hi = (bf16(x).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    if kind != "bf16x3":
        return hi, None
    r = (x.astype(np.float64) - bf16(x)).astype(np.float32)
    lo = (bf16(r).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return hi, lo


def column_exponents(A):
    """e_j with max_i |A(i, j)| 2^-e_j in [2^14, 2^15); 0 for a zero column."""
    mx = np.abs(np.asarray(A, dtype=np.float64)).max(axis=0)
    e = np.zeros(mx.shape, dtype=np.int64)
    nz = mx > 0
    e[nz] = np.floor(np.log2(mx[nz])).astype(np.int64) - 14
    return e


def _gamma(K):
    return 2.0 * K * U32 / (1.0 - K * U32)


def sketch_reference(A, X, kind):
    """(Y_ref, bound) for Y = A X with the operands encoded as for ``kind``."""
    A = np.asarray(A, dtype=np.float32)
    X = np.asarray(X, dtype=np.float32)
    K = A.shape[1]
    if kind == "bf16":
        a, x = bf16(A), bf16(X)
        y, ab = a @ x, np.abs(a) @ np.abs(x)
    elif kind == "bf16x3":
        ah, al = split_bf16(A)
        xh, xl = split_bf16(X)
        y = ah @ xh + ah @ xl + al @ xh
        ab = np.abs(ah) @ np.abs(xh) + np.abs(ah) @ np.abs(xl) + np.abs(al) @ np.abs(xh)
        K = 3 * K
    elif kind == "fp16":
        e = column_exponents(A)
        g = int(e.max())
        a = fp16(A * np.ldexp(1.0, -e)[None, :])
        x = fp16(X * np.ldexp(1.0, e - g)[:, None])
        y, ab = np.ldexp(a @ x, g), np.ldexp(np.abs(a) @ np.abs(x), g)
    else:
        raise ValueError(kind)
    return y, _gamma(K) * ab


def project_reference(A, V, kind):
    """(B_ref, bound) for B = V^T A with the operands encoded as for ``kind``."""
    A = np.asarray(A, dtype=np.float32)
    V = np.asarray(V, dtype=np.float32)
    K = A.shape[0]
    if kind == "bf16":
        a, v = bf16(A), bf16(V)
        b, ab = v.T @ a, np.abs(v).T @ np.abs(a)
    elif kind == "bf16x3":
        ah, al = split_bf16(A)
        vh, vl = split_bf16(V)
        b = vh.T @ ah + vl.T @ ah + vh.T @ al
        ab = np.abs(vh).T @ np.abs(ah) + np.abs(vl).T @ np.abs(ah) + np.abs(vh).T @ np.abs(al)
        K = 3 * K
    elif kind == "fp16":
        e = column_exponents(A)
        a = fp16(A * np.ldexp(1.0, -e)[None, :])
        v = fp16(V)
        sc = np.ldexp(1.0, e)[None, :]
        b, ab = (v.T @ a) * sc, (np.abs(v).T @ np.abs(a)) * sc
    else:
        raise ValueError(kind)
    return b, _gamma(K) * ab
