// Traversal-shape table of a context: which traversal variant to run for a
// cloud of a given mode (one cloud / a batch), dimension and size.  Filled
// by the autotuner (a JSON document, see emst_set_autotune) and consulted
// when the context's traversal is left on "auto".  Host code only.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace emst {

struct TuneEntry {
    int batched;    // 0: emst_build, 1: emst_build_batched
    int dim;        // 2 or 3
    int64_t n_min;  // the entry applies from this many points on
    int variant;
    int lds_depth;  // LDS stack ring entries per lane of variant 13: 4, 8 or 16
};

class TuneTable {
public:
    // Replace the table by the entries of a JSON document
    //   {"entries": [{"mode": "single"|"batched", "dim": 2|3,
    //                 "n_min": <int >= 0>, "variant": <int>,
    //                 "lds_depth": 4|8|16 (optional, default 8)}, ...]}
    // (other keys are ignored).  A variant v is valid if bit v of
    // `valid_variants` is set.  Returns false, leaving the table as it was,
    // on malformed input or out-of-range values; `err` says why.
    bool parse(const char* json, uint32_t valid_variants, std::string* err);
    void clear() { entries_.clear(); }
    // The entry with the largest n_min <= n for (batched, dim), or null if
    // there is none.
    const TuneEntry* pick(int batched, int dim, int64_t n) const;
    std::string dump() const;
    size_t size() const { return entries_.size(); }

private:
    std::vector<TuneEntry> entries_;
};

}  // namespace emst
