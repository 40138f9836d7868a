"""Planted mistakes in the oracle must be caught by its pins.

Each mutant is a one-line textual change to ``oracle/oracle.c`` of the kind a
careless rewrite could make (a dropped term, a wrong sign, a wrong stride or
index, a transposed operand, a wrong rounding rule).  The mutant is compiled
on the CPU into a temporary library and the pin tests of ``test_oracle.py``
are run against it; at least one of them must fail.  Nothing here touches the
GPU or the HIP library."""
import os

import pytest

import oracle
from tests import test_oracle as pins
from tests import test_oracle_int8 as pins8

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = [
    ("drop beta term", "if (beta != 0.0) r = r + beta * c0;", "if (beta != 0.0) r = r;"),
    ("compensation sign", "a->comp += (a->sum - s) + t;", "a->comp += (a->sum - s) - t;"),
    ("compensation dropped at the end", "double ab = compensated ? acc->sum + acc->comp : acc->sum;",
     "double ab = acc->sum;"),
    ("B addressed with A's strides", "ob += idx[l] * p->sB[l];", "ob += idx[l] * p->sA[l];"),
    ("odometer stops one short", "if (++idx[l] < p->ext[l]) break;",
     "if (++idx[l] < p->ext[l] - 1) break;"),
    ("diagonal strides overwritten", "p->sA[slot] += A->strides[d];", "p->sA[slot] = A->strides[d];"),
    ("split drops lo*hi",
     "      acc_add(&acc, (double)xl * (double)yh, compensated);\n    } else if (split == 2) {",
     "    } else if (split == 2) {"),
    ("split keeps lo*lo instead of hi*lo",
     "acc_add(&acc, (double)xh * (double)yl, compensated);\n      acc_add(&acc, (double)xl * (double)yh, compensated);\n    } else if",
     "acc_add(&acc, (double)xl * (double)yl, compensated);\n      acc_add(&acc, (double)xl * (double)yh, compensated);\n    } else if"),
    ("bf16x6 drops m*m", "      acc_add(&acc, (double)xm * (double)ym, compensated);\n", "\n"),
    ("bf16x6 low part from x instead of the residual", "float xl = bf16_rne(xr - xm), yl = bf16_rne(yr - ym);",
     "float xl = bf16_rne(xr), yl = bf16_rne(yr - ym);"),
    ("bf16x6 keeps l*m instead of h*l",
     "acc_add(&acc, (double)xh * (double)yl, compensated);\n      acc_add(&acc, (double)xm * (double)ym, compensated);",
     "acc_add(&acc, (double)xl * (double)ym, compensated);\n      acc_add(&acc, (double)xm * (double)ym, compensated);"),
    ("bf16 truncation instead of RNE", "u += 0x7fffu + keep_odd;", "u += 0u;"),
    ("bf16 ties away from zero", "u += 0x7fffu + keep_odd;", "u += 0x8000u;"),
    ("C0 read when beta == 0", "double c0 = (beta != 0.0) ? c[offC] : 0.0;",
     "double c0 = c[offC];"),
    ("alpha scales C0", "if (beta != 0.0) r = r + beta * c0;", "if (beta != 0.0) r = r + alpha * c0;"),
    ("condition tensor signed", "acc.abssum += fabs(x * y);", "acc.abssum += x * y;"),
    ("output digits row-major", "idx[p.out_lab[m]] = rem % ext;\n      rem /= ext;",
     "idx[p.out_lab[m]] = rem % ext;\n      rem /= (m == 0 ? 1 : ext);"),
    ("alpha ignored", "if (alpha != 0.0) r = alpha * ab;", "if (alpha != 0.0) r = ab;"),
    ("int8 drops the last digit diagonal",
     "for (int j = 1; i + j <= s + 1; ++j) S[i][j] +=", "for (int j = 1; i + j <= s; ++j) S[i][j] +="),
    ("int8 digits truncated instead of rounded", "double q = rint(y);", "double q = trunc(y);"),
    ("int8 scale exponent ignores the 127/128 limit", "return f <= 127.0 / 128.0 ? e : e + 1;", "return e;"),
    ("int8 scale exponent one too large", "return f <= 127.0 / 128.0 ? e : e + 1;",
     "return f <= 127.0 / 128.0 ? e + 1 : e + 2;"),
    ("int8 digits in base 2^8", "double y = ldexp(r, 7);", "double y = ldexp(r, 8);"),
    ("int8 B sliced with A's scale", "int8_digits(b[offB], eb, s, db);", "int8_digits(b[offB], ea, s, db);"),
    ("int8 pair weight off by one digit", "ldexp((double)S[i][j], -7 * (i + j))",
     "ldexp((double)S[i][j], -7 * (i + j - 1))"),
    ("int8 row and column scales dropped", "return ldexp(acc.sum + acc.comp, ea + eb);",
     "return acc.sum + acc.comp;"),
    ("int8 non-finite rows not flagged", "if (!finite) return NAN;", "if (0) return NAN;"),
    ("int8 row max over B", "if (fabs(x) > amax) amax = fabs(x);", "if (fabs(y) > amax) amax = fabs(y);"),
]

CHECKS = [
    lambda: [pins.test_bruteforce_integer_exact(None, s) for s in range(24)],
    lambda: [pins.test_bruteforce_real(None, s) for s in range(6)],
    lambda: pins.test_kronecker_delta_closed_form(None),
    lambda: pins.test_all_ones_closed_form(None),
    lambda: pins.test_ones_times_random_is_marginal(None),
    lambda: [pins.test_agrees_with_permuted_gemm(None, s) for s in range(4)],
    lambda: pins.test_permuted_gemm_integer_exact(None),
    lambda: pins.test_blas_conventions_nan(None),
    lambda: pins.test_empty_sum_and_empty_output(None),
    lambda: pins.test_compensated_summation(None),
    lambda: pins.test_condition_tensor_mixed_signs(None),
    lambda: pins.test_bf16_rne_matches_torch(None),
    lambda: pins.test_split_reference_matches_library_split(None),
    lambda: pins.test_split_exact_when_inputs_are_bf16(None),
    lambda: pins.test_bf16x6_split_matches_library_split(None),
    lambda: pins.test_bf16x6_error_bound(None),
    lambda: pins.test_golden_fixtures(None),
    lambda: pins8.test_digits_definition(None),
    lambda: [pins8.test_bruteforce_exact_rational(None, s) for s in range(8)],
    lambda: [pins8.test_integer_inputs_exact(None, s) for s in range(4)],
    lambda: pins8.test_kronecker_closed_form(None),
    lambda: pins8.test_power_of_two_scaling(None),
    lambda: pins8.test_error_bound_and_convergence(None),
    lambda: pins8.test_nonfinite_rows_give_nan(None),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, monkeypatch, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not unique/present: " + name
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    lib_path = oracle.build(force=True, src=str(mpath), out=str(tmp_path / "libmutant.so"))
    lib = oracle.load(lib_path)
    monkeypatch.setattr(oracle, "load", lambda path=None: lib)
    failures = 0
    for chk in CHECKS:
        try:
            chk()
        except (AssertionError, oracle.OracleError):
            failures += 1
    assert failures > 0, "no pin caught mutant: " + name
