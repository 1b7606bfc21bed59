// Launch-shape knobs chosen by the project's autotuner (paper_1901_10559_amd/tune.py).
// Each knob has a name and an integer value; the values the tuner measured
// best on the device are compiled in from tuned_table.inc, and
// ids_tune_set overrides them at run time (the tuner tries its candidates
// that way).
#pragma once
#include <stdint.h>

#include <string>

namespace ids {

// value of knob `key` (the tuned table's, or an override); `dflt` if the key
// is unknown
int64_t tune_get(const std::string& key, int64_t dflt);

// "n1k" / "n4k" / "n16k" / "ninf": the column-count bucket of the select knobs
inline const char* n_bucket(int64_t n) {
    return n <= 1024 ? "n1k" : n <= 4096 ? "n4k" : n <= 16384 ? "n16k" : "ninf";
}

}  // namespace ids
