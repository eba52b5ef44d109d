"""Each pin of tests/_pins.py catches the mistakes it is meant to catch: a
copy of the oracle's sources with one planted mistake (sign, lever arm,
transposed inertia, dropped term of the implicit PD drive, wrong derivative
rule, missing cap ...; tests/_mutants.py) is built, and the named pins must
fail on it while they pass on the oracle itself (test_oracle_pins.py)."""
import concurrent.futures as cf
import os

import pytest

import oracle
import _pins
from _mutants import MUTANTS


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory):
    base = oracle.source_texts()
    root = tmp_path_factory.mktemp("oracle_mutants")

    def build(name):
        fname, old, new, _ = MUTANTS[name]
        texts = dict(base)
        assert texts[fname].count(old) == 1, f"{name}: the planted text must occur once in {fname}"
        texts[fname] = texts[fname].replace(old, new)
        return name, oracle.build_variant(texts, os.path.join(str(root), name))

    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        return dict(ex.map(build, MUTANTS))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(mutant_libs, name):
    path = mutant_libs[name]

    def mk(b, **kw):
        return oracle.Oracle(b, lib_path=path, **kw)

    for pin_name in MUTANTS[name][3]:
        with pytest.raises(AssertionError):
            getattr(_pins, pin_name)(mk)
