"""Host references for the low-precision storage formats (test helpers).

bfloat16 rounding comes from torch's CPU conversion; FP8 e4m3 (OCP
"e4m3fn": 1 sign, 4 exponent bits with bias 7, 3 mantissa bits, no
infinities, largest finite 448, subnormals k * 2^-9) is decoded from its bit
layout and rounded to the nearest code, ties to the even code."""
import numpy as np


def e4m3_table():
    vals = np.zeros(256)
    for code in range(256):
        sgn = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        m = code & 0x7
        if e == 0xF and m == 0x7:
            vals[code] = np.nan
        elif e == 0:
            vals[code] = sgn * m * 2.0 ** -9
        else:
            vals[code] = sgn * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return vals


_TAB = e4m3_table()


def e4m3_encode(x):
    """Nearest e4m3 code of each value (saturating at +-448), ties to even."""
    x = np.clip(np.asarray(x, np.float64), -448.0, 448.0)
    finite = np.where(np.isnan(_TAB), np.inf, _TAB)
    out = np.empty(x.shape, np.uint8)
    flat = x.ravel()
    res = out.ravel()
    for idx, v in enumerate(flat):
        d = np.abs(finite - v)
        best = np.flatnonzero(d == d.min())
        if len(best) > 1:
            # prefer the code with the same sign as v (for +-0), then even LSB
            same = [c for c in best if (c >= 128) == (np.signbit(v))]
            best = same or list(best)
            even = [c for c in best if c % 2 == 0]
            best = even or best
        res[idx] = best[0]
    return out


def e4m3_decode(codes):
    return _TAB[np.asarray(codes, np.uint8)]


def bf16_round(x):
    import torch
    return torch.from_numpy(np.asarray(x, np.float32)).to(torch.bfloat16).to(torch.float32).numpy()
