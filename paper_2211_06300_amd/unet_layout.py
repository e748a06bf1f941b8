"""Layer layout of the preconditioner network, as include/esi.h states it:
the flat parameter vector holds, per layer in this order, its weights then its
bias.  Used to initialise parameters and to index them by layer."""

# (name, kind, cin, cout); kind: "c3" 3x3 conv [co][ci][3][3], "t2" 2x2
# transposed conv [ci][co][2][2], "c1" 1x1 conv [co][ci]
LAYERS = [
    ("c1a", "c3", 3, 16), ("c1b", "c3", 16, 16), ("c2a", "c3", 16, 32), ("c2b", "c3", 32, 32),
    ("c3a", "c3", 32, 64), ("c3b", "c3", 64, 64), ("c4a", "c3", 64, 128), ("c4b", "c3", 128, 128),
    ("u3", "t2", 128, 64), ("d3a", "c3", 128, 64), ("d3b", "c3", 64, 64),
    ("u2", "t2", 64, 32), ("d2a", "c3", 64, 32), ("d2b", "c3", 32, 32),
    ("u1", "t2", 32, 16), ("d1a", "c3", 32, 16), ("d1b", "c3", 16, 16),
    ("out", "c1", 16, 1),
]

_TAPS = {"c3": 9, "t2": 4, "c1": 1}


def fan_segments():
    """(weight count, fan-in, bias count) per layer."""
    out = []
    for _, kind, ci, co in LAYERS:
        fan = ci * (9 if kind == "c3" else 1)
        out.append((_TAPS[kind] * ci * co, fan, co))
    return out


def num_params() -> int:
    return sum(n + b for n, _, b in fan_segments())
