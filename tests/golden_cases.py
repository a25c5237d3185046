"""Parser for tests/golden/stream_cases.txt (hand-written compressed-stream fixtures)."""

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load_stream_cases(path=None):
    path = path or os.path.join(HERE, "golden", "stream_cases.txt")
    cases = []
    cur = None
    repeat = 1
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            key = tok[0]
            if key == "case":
                cur = {"name": tok[1], "particles": []}
                repeat = 1
            elif key == "end":
                n_c = cur["n_c"]
                pb = cur.get("widths", (1, 2))[0]
                S = (256 ** pb) * n_c
                P = np.array(cur["particles"], dtype=np.float64).reshape(-1, 6)
                cur["x"] = (P[:, :3] / S).astype(np.float32)
                cur["v"] = P[:, 3:].astype(np.float32)
                cases.append(cur)
                cur = None
            elif key in ("n_c", "brick"):
                cur[key] = int(tok[1])
            elif key == "widths":
                cur["widths"] = (int(tok[1]), int(tok[2]))
            elif key == "repeat":
                repeat = int(tok[1])
            elif key == "particle":
                vals = [float(t) for t in tok[1:]]
                for _ in range(repeat):
                    cur["particles"].append(vals)
                repeat = 1
            elif key in ("counts", "keys"):
                cur[key] = [int(t) for t in tok[1:]]
            elif key in ("body", "body_prefix", "record"):
                cur[key] = bytes(int(t, 16) for t in tok[1:])
            else:
                raise ValueError(f"unknown fixture line: {line}")
    return cases
