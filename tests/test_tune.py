"""The launch-plan autotuner's host logic and the committed table it writes (CPU only).

The kernels of a colour take their launch plan from a table indexed by the colour's box
count; `tune.py` measures candidates per field and writes the table.  Pinned here: the bucket
of a box count, the bucket of a level (its largest colour under the 3 x 3 colouring), the
RSS_TUNE string, and that the committed table has the tuner's buckets, one value per field and
only values the tuner could have chosen (its candidates or its defaults).
"""
import os
import re

from paper_1609_08130_amd import tune

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "..", "paper_1609_08130_amd", "csrc", "tuned_plans.inc")


def test_bucket_bounds():
    assert [tune.bucket_of(n) for n in (1, 63, 64, 255, 256, 511, 512, 1023, 1024, 10 ** 6)] == \
        [0, 0, 1, 1, 2, 2, 3, 3, 4, 4]


def test_level_bucket_is_the_largest_colour():
    # depth d: 2^d boxes a side, colour classes of ceil(2^d / 3)^2 boxes at most
    for d in range(2, 11):
        nb = 2 ** d
        largest = max(len(range(cx, nb, 3)) * len(range(cy, nb, 3)) for cx in range(3) for cy in range(3))
        assert tune.level_bucket(d) == tune.bucket_of(largest), d
    assert [tune.level_bucket(d) for d in (2, 3, 4, 5, 6, 7)] == [0, 0, 0, 1, 2, 4]


def test_tune_string_names_every_bucket_and_field():
    table = [[10 * b + i for i in range(len(tune.FIELDS))] for b in range(len(tune.BUCKET_LO))]
    items = tune.env_of(table).split(",")
    assert len(items) == len(tune.BUCKET_LO) * len(tune.FIELDS)
    for b in range(len(tune.BUCKET_LO)):
        for i, f in enumerate(tune.FIELDS):
            assert f"b{b}.{f}={10 * b + i}" in items


def _read_table(path):
    text = open(path).read()
    lo = re.search(r"kPlanBucketLo\[kPlanBuckets\] = \{([^}]*)\}", text).group(1)
    rows = re.findall(r"\{([0-9, ]+)\},", text.split("kPlanTable")[1])
    return [int(v) for v in lo.split(",")], [[int(v) for v in r.split(",")] for r in rows]


def test_committed_table_is_in_the_tuners_space(tmp_path):
    lo, rows = _read_table(TABLE)
    assert lo == tune.BUCKET_LO
    assert len(rows) == len(tune.BUCKET_LO)
    for b, row in enumerate(rows):
        assert len(row) == len(tune.FIELDS)
        for i, f in enumerate(tune.FIELDS):
            cands, _ = tune.CANDIDATES[f]
            assert row[i] in cands or row[i] == tune.DEFAULTS[b][i], (b, f, row[i])
    # what write_table writes reads back the same
    out = tmp_path / "plans.inc"
    tune.write_table(str(out), rows, "test")
    assert _read_table(str(out)) == (lo, rows)


def test_tolerances_weigh_the_same():
    # two tolerances, one 10x slower overall: a value 10% faster at the slow one and 10%
    # slower at the fast one scores the same as the starting value
    base = {1e-6: {0: 10.0, 4: 20.0}, 1e-9: {0: 100.0, 4: 200.0}}
    same = tune.combine(base, base)
    assert same == {0: 2.0, 4: 2.0}
    mixed = tune.combine({1e-6: {0: 11.0, 4: 20.0}, 1e-9: {0: 90.0, 4: 200.0}}, base)
    assert abs(mixed[0] - 2.0) < 1e-12 and mixed[4] == 2.0


def test_bucket_times_sum_the_levels_of_a_bucket():
    # depths 2, 3, 4 share bucket 0; depth 7 is bucket 4; phases (ID, elimination, Schur)
    med = {(2, "strong"): (1.0, 2.0, 3.0), (3, "strong"): (1.0, 2.0, 3.0), (4, "strong"): (1.0, 2.0, 3.0),
           (7, "strong"): (5.0, 6.0, 7.0)}
    assert tune.bucket_times(med, 0) == {0: 3.0, 4: 5.0}
    assert tune.bucket_times(med, 2) == {0: 9.0, 4: 7.0}
