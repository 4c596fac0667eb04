"""Each plausible mistake planted in the oracle is caught by some pin.

The mistakes are planted on the CPU only, in temporary copies of the oracle
source; the real oracle is never modified.  A mutant survives if every pin in
``oracle_pins.ALL_PINS`` still passes, which would mean the pins cannot tell
that mistake from the correct code.
"""
import os

import pytest

import oracle
import oracle_pins

MUTANTS = [
    ("dropped last coordinate",
     "for (int k = 0; k < E; ++k) {\n        float diff",
     "for (int k = 0; k < E - 1; ++k) {\n        float diff"),
    ("lag ignores tau",
     "Sf[ti - (int64_t)k * tau] - Sf[tj - (int64_t)k * tau]",
     "Sf[ti - (int64_t)k] - Sf[tj - (int64_t)k]"),
    ("unfused accumulate", "acc = fmaf(diff, diff, acc);", "acc = diff * diff + acc;"),
    ("ties to higher index", "(a.d2 == b.d2 && a.j < b.j)", "(a.d2 == b.d2 && a.j > b.j)"),
    ("E neighbours instead of E+1", "const int k = E + 1;\n    int n = 0;",
     "const int k = E;\n    int n = 0;"),
    ("weights not scaled by d_1", "u[m] = exp(-d[m] / d[0]);", "u[m] = exp(-d[m]);"),
    ("weights from squared distance", "d[m] = sqrt((double)best[m].d2);",
     "d[m] = (double)best[m].d2;"),
    ("weights not normalised", "p += (u[m] / su) * T[best[m].j + off];",
     "p += u[m] * T[best[m].j + off];"),
    ("target not lag aligned", "p += (u[m] / su) * T[best[m].j + off];",
     "p += (u[m] / su) * T[best[m].j];"),
    ("observed not lag aligned", "O[q] = T[i + off];", "O[q] = T[i];"),
    ("self not excluded", "return d <= excl;", "return d < excl;"),
    ("zero-distance rule", "u[m] = (d[m] == 0.0) ? 1.0 : 0.0;", "u[m] = 1.0;"),
    ("pearson without sqrt", "return sab / sqrt(saa * sbb);", "return sab / (saa * sbb);"),
    ("pearson mean over n-1", "ma /= (double)n;", "ma /= (double)(n - 1);"),
    ("sampler off by one", "if (u < (uint64_t)(L_eff - s))", "if (u <= (uint64_t)(L_eff - s))"),
    ("sampler key drops tau",
     "    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)tau);\n    s = oracle_sm64_mix(s ^ (uint64_t)L_eff);",
     "    s = oracle_sm64_mix(s ^ (uint64_t)L_eff);"),
    ("nested shuffle range one short", "(unsigned __int128)z * (uint64_t)(N_e - k);",
     "(unsigned __int128)z * (uint64_t)(N_e - k - 1);"),
    ("nested key drops r",
     "    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)r_index);\n    return s;\n}\n\n/*\n * First n_out",
     "    return s;\n}\n\n/*\n * First n_out"),
    ("shared E without the shift", "const int64_t d = (int64_t)(Emax - Es[e]) * tau;",
     "const int64_t d = 0;"),
    ("shared library keyed by E", "oracle_sample_library(seed, 0, tau, le, q, Nc, lib);",
     "oracle_sample_library(seed, Emax, tau, le, q, Nc, lib);"),
    ("nested library is a suffix", "st = oracle_neighbors(Y, X, N, E, tau, perm, le,",
     "st = oracle_neighbors(Y, X, N, E, tau, perm + (Lmax - le), le,"),
    ("splitmix constant", "0xbf58476d1ce4e5b9ULL", "0xbf58476d1ce4e5b8ULL"),
    ("sampler key folds tau before E",
     "    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)E);\n    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)tau);\n    s = oracle_sm64_mix(s ^ (uint64_t)L_eff);",
     "    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)tau);\n    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)E);\n    s = oracle_sm64_mix(s ^ (uint64_t)L_eff);"),
    ("sampler key folds r twice",
     "    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)r_index);\n    return s;\n}\n\n/*\n * Selection",
     "    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)r_index);\n    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)r_index);\n    return s;\n}\n\n/*\n * Selection"),
    ("sampler draw without the gamma step", "    *state += 0x9e3779b97f4a7c15ULL;\n", "    *state ^= 0x9e3779b97f4a7c15ULL;\n"),
    ("clamp one short", "const int64_t Le = L < Ne ? L : Ne;",
     "const int64_t Le = L < Ne ? L : Ne - 1;"),
    ("query set ignored", "const int64_t i = query_set ? lib[q] : q;", "const int64_t i = q;"),
]


@pytest.fixture(scope="module")
def source():
    with open(oracle.SOURCE) as f:
        return f.read()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, source, name, old, new):
    assert source.count(old) == 1, f"mutation site for '{name}' not unique"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new))
    so = str(tmp_path / "libmutant.so")
    oracle.compile_oracle(str(src), so)
    orc = oracle.Oracle(so)
    caught = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(orc)
        except (AssertionError, oracle.OracleError, ValueError, IndexError):
            caught.append(pin.__name__)
            break
    assert caught, f"mutant '{name}' passes every pin"
    os.remove(so)
