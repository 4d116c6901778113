"""Writes the stored expected values under tests/golden/ from the FP64 oracle.

Run from the repository root:  python tests/golden/make_golden.py
Only ``oracle`` and ``workloads`` are used; nothing here touches the HIP library.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main():
    sq = W.square_array(1, 1, 0.03, 0.0, 32)
    pair = W.square_array(2, 1, 0.03, 0.035, 32)
    circ = W.single_circle(0.05, 64, 1e-3, 0.5)
    out = {
        "_source": "oracle.inductance_matrix[_fast]; regenerate with tests/golden/make_golden.py",
        "square_3cm_a1mm_self_H": float(O.inductance_matrix_fast(sq.verts, sq.seg_off, sq.wire_a)[0, 0]),
        "square_3cm_pitch35mm_mutual_H": float(O.inductance_matrix_fast(pair.verts, pair.seg_off, pair.wire_a)[0, 1]),
        "polygon64_r5cm_a1mm_self_H": float(O.inductance_matrix(circ.verts, circ.seg_off, circ.wire_a)[0, 0]),
        "maxwell_coaxial_r5cm_d1mm_H": float(O.coaxial_circles_mutual(0.05, 0.05, 1e-3)),
    }
    with open(os.path.join(HERE, "inductance.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
