"""Plants plausible mistakes in copies of the oracle (on the CPU) and checks
that the pins catch every one: a pin suite that passes a broken oracle would
not be pinning anything."""

import os

import pytest

import oracle
from pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.cpp")

# (name, text in oracle.cpp, replacement)
MUTANTS = [
    ("lt_becomes_le", "case OC_LT: return v < lo;", "case OC_LT: return v <= lo;"),
    ("range_upper_inclusive", "default: return lo <= v && v < hi;", "default: return lo <= v && v <= hi;"),
    ("ne_becomes_eq", "case OC_NE: return v != lo;", "case OC_NE: return v == lo;"),
    ("i8_read_unsigned", "case OT_I8: return static_cast<const int8_t*>(col)[i];",
     "case OT_I8: return static_cast<const uint8_t*>(col)[i];"),
    ("selection_ignored", "int64_t row = sel ? static_cast<int64_t>(sel[i]) : i;", "int64_t row = i;"),
    ("join_drops_duplicate_build_keys",
     "for (int64_t b = 0; b < nb; ++b) table[read_value(build, key_type, b)].push_back(static_cast<uint32_t>(b));",
     "for (int64_t b = 0; b < nb; ++b) { auto& v = table[read_value(build, key_type, b)]; if (v.empty()) v.push_back(static_cast<uint32_t>(b)); }"),
    ("join_pairs_swapped", "out_build[count] = b;", "out_build[count] = static_cast<uint32_t>(p);"),
    ("min_starts_at_zero", "int64_t min = std::numeric_limits<int64_t>::max();", "int64_t min = 0;"),
    ("sum_of_magnitudes", "sum += static_cast<uint64_t>(v);", "sum += static_cast<uint64_t>(v < 0 ? -v : v);"),
    ("avg_off_by_one_count", "/ static_cast<double>(count);", "/ static_cast<double>(count + 1);"),
    ("avg_integer_division", "double avg = static_cast<double>(static_cast<int64_t>(sum)) / static_cast<double>(count);",
     "double avg = static_cast<double>(static_cast<int64_t>(sum) / count);"),
    ("groups_sorted_descending", "return *a < *b; });", "return *a > *b; });"),
    ("pipeline_second_dim_ignored", "for (uint32_t b1 : *match[1]) {", "for (uint32_t b1 : no_dim) {"),
    ("pipeline_unmatched_rows_kept", "dropped = true;\n        break;", "continue;"),
    ("pipeline_filter_ignored", "if (!pred.holds(fact, fact_types, i)) continue;", ""),
    ("semi_join_keeps_misses", "if (keys.count(read_value(probe, key_type, p))) out[written++]",
     "if (!keys.count(read_value(probe, key_type, p))) out[written++]"),
    ("gather_reads_row_id", "out[i] = read_value(col, type, idx[i]);", "out[i] = read_value(col, type, i);"),
    ("topn_ascending_when_desc", "return desc ? gt : lt;", "return desc ? lt : gt;"),
    ("topn_ties_by_position", "if (keys[k][a] != keys[k][b]) return keys[k][a] < keys[k][b];", ""),
    ("topn_drops_last", "for (int64_t i = 0; i < m; ++i) out[i] = rows[i];",
     "for (int64_t i = 0; i < m; ++i) out[i] = rows[i + (i + 1 == m && m < n ? 1 : 0)];"),
    ("string_groups_ignore_int_key", "const int64_t k2 = ikey_type ? read_value(ikey, ikey_type, i) : 0;",
     "const int64_t k2 = 0;"),
    ("string_keys_truncated", "static_cast<size_t>(offsets[i + 1] - offsets[i]));",
     "static_cast<size_t>(std::min<int64_t>(offsets[i + 1] - offsets[i], 2)));"),
    ("string_group_last_row", "auto it = groups.find({key, k2});\n    if (it == groups.end()) {",
     "auto it = groups.find({key, k2});\n    if (it != groups.end()) it->second.first = static_cast<uint32_t>(i);\n    if (it == groups.end()) {"),
    ("ungrouped_empty_has_no_row", "if (nkeys == 0) groups[std::vector<int64_t>()].resize(naggs);\n  std::vector<int64_t> key(nkeys);\n  for (int64_t i = 0; i < n; ++i) {\n    for (int k",
     "std::vector<int64_t> key(nkeys);\n  for (int64_t i = 0; i < n; ++i) {\n    for (int k"),
]


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, source, name, old, new):
    assert source.count(old) == 1, f"mutation site for {name} not found exactly once"
    src = tmp_path / "mutant.cpp"
    src.write_text(source.replace(old, new))
    lib = oracle.build(str(src), str(tmp_path / "libmutant.so"))
    mutant = oracle.Oracle(lib)
    caught = []
    for pin in ALL_PINS:
        try:
            pin(mutant)
        except AssertionError:
            caught.append(pin.__name__)
        except (IndexError, ValueError) as e:  # malformed output also exposes the mutant
            caught.append(f"{pin.__name__} ({type(e).__name__})")
    assert caught, f"no pin catches the mutant {name}"
