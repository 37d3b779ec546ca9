"""The row-mapping candidates of the autotuner satisfy the constraints the
kernels assert at build time (lanes per row a power of two up to 32 and at
least the chunks per row; rounds in flight at least one), for every block
width and element size the library instantiates."""
from paper_2112_07862_amd import tune


def test_candidates_build_time_constraints():
    assert "default" in tune.CANDIDATES
    for name, c in tune.CANDIDATES.items():
        lanes1, epl, unr1, unr = c
        for size, kbs in ((2, (8, 16)), (4, (4, 8, 16)), (8, (4, 8, 16))):  # FP16, FP32, FP64
            for kb in kbs:
                nch = kb * size // 16
                g = lanes1 if nch == 1 else epl * nch
                assert g >= nch and g <= 32 and g & (g - 1) == 0, (name, size, kb, g)
                assert (unr1 if nch == 1 else unr) >= 1, name
        assert len(tune.defines(c)) == 4


def test_default_candidate_matches_library_defaults():
    import re
    import os
    src = open(os.path.join(os.path.dirname(tune.__file__), "csrc", "rowops.h")).read()
    got = {m.group(1): int(m.group(2))
           for m in re.finditer(r"#define (ME_ROW_\w+) (\d+)", src)}
    want = dict(d.split("=") for d in tune.defines(tune.CANDIDATES["default"]))
    assert {k: int(v) for k, v in want.items()} == got
