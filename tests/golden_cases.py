"""Parser for tests/golden/hand_cases.txt (test-only)."""
import os

import numpy as np

from paper_1704_00878_amd import synth

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_cases.txt")


def load():
    cases, cur = [], None
    with open(PATH) as fh:
        for raw in fh:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            if key in ("case", "msa"):
                cur = {"kind": key, "name": vals[0]}
                cases.append(cur)
            else:
                cur[key] = vals
    out = []
    for c in cases:
        d = {"kind": c["kind"], "name": c["name"], "go": int(c["go"][0]), "ge": int(c["ge"][0])}
        if c["kind"] == "case":
            d["center"] = synth.encode(c["center"][0])
            d["seq"] = synth.encode(c["seq"][0])
            d["score"] = int(c["score"][0])
            d["cells"] = tuple(int(x) for x in c["cells"])
            d["ops"] = c["ops"][0]
            d["ins"] = np.array([int(x) for x in c["ins"]], np.uint16)
            d["aligned"] = np.array([int(x) for x in c["aligned"]], np.uint8)
        else:
            d["seqs"] = [synth.encode(x) for x in c["seqs"]]
            d["center"] = int(c["center"][0])
            d["G"] = np.array([int(x) for x in c["G"]], np.int32)
            d["rows"] = c["rows"]
            d["sp"] = int(c["sp"][0])
            d["sp_blosum"] = int(c["sp_blosum"][0])
        out.append(d)
    return out


def row_text(msa_row) -> str:
    return synth.decode(msa_row)
