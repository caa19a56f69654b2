"""The pins have teeth: each plausible mistake planted in a copy of the
oracle (a wrong constant, rotation or index, a dropped or flipped condition,
an off-by-one) makes at least one oracle pin test fail.  Runs on the CPU only;
the real oracle is untouched."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_TESTS = ["tests/test_oracle_xxh64.py", "tests/test_oracle_snapshot.py", "tests/test_oracle_compare.py",
             "tests/test_oracle_graph.py", "tests/test_oracle_region.py", "tests/test_oracle_ragged.py",
             "tests/test_oracle_units.py", "tests/test_golden.py"]

MUTANTS = {
    "round uses P1": ("acc = acc + lane * PRIME2;", "acc = acc + lane * PRIME1;"),
    "round rotation 33": ("acc = rotate_left(acc, 31);", "acc = rotate_left(acc, 33);"),
    "merge rotation": ("rotate_left(v2, 7)", "rotate_left(v2, 8)"),
    "tail lane constant": ("acc = rotate_left(acc, 27) * PRIME1 + PRIME4;", "acc = rotate_left(acc, 27) * PRIME1 + PRIME3;"),
    "avalanche shift": ("acc ^= acc >> 29;", "acc ^= acc >> 28;"),
    "zero test skips last byte": ("for (uint64_t i = 0; i < len; ++i)", "for (uint64_t i = 0; i + 1 < len; ++i)"),
    "partial page hashed whole": ("hash[g] = kco_xxh64(page, len, seed);", "hash[g] = kco_xxh64(page, unit, seed);"),
    "partial slot not padded": ("memset(packed + slot * unit + len, 0, unit - len);", ""),
    "restore writes whole page": ("memcpy(host_ptr[a] + p * unit, packed + s * unit, page_len(&ranges[a], p, unit));",
                                  "memcpy(host_ptr[a] + p * unit, packed + s * unit, unit);"),
    "units counted as pages": ("pages += (size + unit - 1) / unit;", "pages += (size + PAGE - 1) / PAGE;"),
    "unit stride taken as the page": ("const uint8_t *page = host_ptr[a] + p * unit;",
                                      "const uint8_t *page = host_ptr[a] + p * PAGE;"),
    "restore accepts a VA inside a unit": ("if (a < 0 || (va - ranges[a].base) % unit != 0) {", "if (a < 0) {"),
    "range scan skips its first word": ("for (uint64_t off = 0; off + 8 <= ranges[a].size; off += 8) {\n"
                                        "    uint64_t w = read_u64_le(host + off);",
                                        "for (uint64_t off = 8; off + 8 <= ranges[a].size; off += 8) {\n"
                                        "    uint64_t w = read_u64_le(host + off);"),
    "scan reads a straddling word": ("for (uint64_t off = 0; off + 8 <= ranges[a].size; off += 8) { /* words wholly inside */\n"
                                     "      uint64_t w = read_u64_le(host_ptr[a] + off);\n      res->n_words += 1;",
                                     "for (uint64_t off = 0; off < ranges[a].size; off += 8) { /* words wholly inside */\n"
                                     "      uint64_t w = read_u64_le(host_ptr[a] + off);\n      res->n_words += 1;"),
    "changed inverted": ("if (prior && hash[g] != prior[g])", "if (prior && hash[g] == prior[g])"),
    "page VA off by one page": ("page_va[slot] = ranges[a].base + p * unit;", "page_va[slot] = ranges[a].base + (p + 1) * unit;"),
    "delta keep uses or": ("if (changed_bm != NULL) keep = keep && bit_get(changed_bm, g);",
                           "if (changed_bm != NULL) keep = keep || bit_get(changed_bm, g);"),
    "window upper edge inclusive": ("      if (w < win_lo || w >= win_hi) continue;",
                                    "      if (w < win_lo || w > win_hi) continue;"),
    "range scan window lower edge exclusive": ("    if (w < win_lo || w >= win_hi) continue;\n    res->n_ptr_like",
                                               "    if (w <= win_lo || w >= win_hi) continue;\n    res->n_ptr_like"),
    "range end inclusive": ("if (va - ranges[lo].base < ranges[lo].size) return (int64_t)lo;",
                            "if (va - ranges[lo].base <= ranges[lo].size) return (int64_t)lo;"),
    "adjacent ranges rejected": ("if (base < prev_end) return KCO_EORDER;", "if (base <= prev_end) return KCO_EORDER;"),
    "window margin 2 GiB": ("const uint64_t margin = 1ULL << 32;", "const uint64_t margin = 1ULL << 31;"),
    "ulp ignores cand sign": ("int sc = (cand_bits & sb) != 0,", "int sc = 0,"),
    "log bins shifted": ("return 12u + k < 47u ? 12u + k : 47u;", "return 11u + k < 47u ? 11u + k : 47u;"),
    "rel includes zero golds": ("if (vg != 0.0 && !is_inf_value(dtype, vg)) {", "if (!is_inf_value(dtype, vg)) {"),
    "last mismatch kept": ("if (res->first_mismatch == UINT64_MAX) res->first_mismatch = i;", "res->first_mismatch = i;"),
    "byte count per element": ("if (pc[b] != pg[b]) res->n_mismatch_bytes += 1;", "res->n_mismatch_bytes += 1;"),
    "NaN payloads split both-NaN": ("if (nan_c && nan_g) {", "if (nan_c && nan_g && c == g) {"),
    "fp16 exponent bias": ("small_float(e, m, 10, 15)", "small_float(e, m, 10, 14)"),
    "subnormal scale": ("if (e == 0) return ldexp((double)m, 1 - bias - mbits);",
                        "if (e == 0) return ldexp((double)m, -bias - mbits);"),
    "e4m3fnuz bias 7": ("small_float((uint32_t)mag >> 3, (uint32_t)mag & 0x7u, 3, 8)",
                        "small_float((uint32_t)mag >> 3, (uint32_t)mag & 0x7u, 3, 7)"),
    "e5m2fnuz bias 15": ("small_float((uint32_t)mag >> 2, (uint32_t)mag & 0x3u, 2, 16)",
                         "small_float((uint32_t)mag >> 2, (uint32_t)mag & 0x3u, 2, 15)"),
    "e5m2 without infinities": ("v = e == 31 ? INFINITY : small_float(e, m, 2, 15);", "v = small_float(e, m, 2, 15);"),
    "fnuz NaN by magnitude": ("case KCO_FP8_E4M3FNUZ: case KCO_FP8_E5M2FNUZ: return bits == 0x80u;",
                              "case KCO_FP8_E4M3FNUZ: case KCO_FP8_E5M2FNUZ: return mag == 0x7Fu;"),
    "f64 inf taken for NaN": ("case KCO_F64: return mag > 0x7FF0000000000000ULL;",
                              "case KCO_F64: return mag >= 0x7FF0000000000000ULL;"),
    "integers not sign-extended": ("if ((c >> (nb - 1)) & 1u) c |= ~0ULL << nb;", ""),
    "integer order unsigned": ("*dist = ci >= gi ? c - g : g - c;", "*dist = c >= g ? c - g : g - c;"),
    "integer error by fp64 subtraction": ("abs_err = (double)d; /* exact difference, one rounding */",
                                          "abs_err = fabs(vc - vg);"),
    "tolerance inclusive": ("if (d > ulp_tol) res->n_over_tol += 1;", "if (d >= ulp_tol) res->n_over_tol += 1;"),
    "rtol scales the candidate": ("close = abs_err <= atol + rtol * fabs(vg);", "close = abs_err <= atol + rtol * fabs(vc);"),
    "infinities always close": ("close = vc == vg;", "close = 1;"),
    "edge points back to its source": ("if (b >= 0) bit_set(edge_bm + (uint64_t)a * rw, (uint64_t)b);",
                                       "if (b >= 0) bit_set(edge_bm + (uint64_t)a * rw, (uint64_t)a);"),
    "graph ignores the window": ("if (!(w >= win_lo && w < win_hi)) continue; /* not pointer-like */", ""),
    "reach follows edges backwards": ("if (bit_get(edge_bm + (uint64_t)a * rw, b) && !bit_get(reach_bm, b)) {",
                                      "if (bit_get(edge_bm + (uint64_t)b * rw, a) && !bit_get(reach_bm, b)) {"),
    "roots not expanded": ("queue[tail++] = (uint32_t)r;", "(void)0;"),
    "zero pages take a snapshot slot": ("      const uint8_t *gold = NULL; /* NULL: the golden unit is all zeros */\n",
                                        "      const uint8_t *gold = NULL; /* NULL: the golden unit is all zeros */\n"
                                        "      if (bit_get(gold_zero_bm, g)) ++slot;\n"),
    "diff pages counted per byte": ("if (d > 0) res[a].n_diff_pages += 1;", "res[a].n_diff_pages += d;"),
    "page VA not checked": ("if (s >= n_valid || gold_page_va[s] != va) {", "if (s >= n_valid) {"),
}


def _run_mutant(name, tmp):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "kco.c")).read()
    assert src.count(old) == 1, f"mutant {name!r}: pattern not unique"
    d = os.path.join(tmp, "m%d" % list(MUTANTS).index(name))
    os.makedirs(d, exist_ok=True)
    shutil.copy(os.path.join(ROOT, "oracle", "kco.h"), d)
    with open(os.path.join(d, "kco.c"), "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(d, "libkco.so")
    subprocess.run(["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-o", lib,
                    os.path.join(d, "kco.c"), "-lm"], check=True, capture_output=True)
    env = dict(os.environ, KCO_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *PIN_TESTS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode


def test_every_mutant_is_caught(tmp_path, oracle_lib):
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        codes = dict(zip(MUTANTS, ex.map(lambda n: _run_mutant(n, str(tmp_path)), MUTANTS)))
    survived = [n for n, c in codes.items() if c == 0]
    assert not survived, f"mutants not caught by any pin: {survived}"
    assert all(c == 1 for c in codes.values()), codes   # failures, not crashes or collection errors
