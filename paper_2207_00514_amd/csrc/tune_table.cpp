// Parser, lookup and serialisation of the traversal-shape table.  The JSON
// reader accepts exactly the document shape the autotuner writes: objects,
// arrays, strings without escapes other than \" and \\, integers, and the
// literals true / false / null.
#include "tune_table.h"

#include <ctype.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

namespace emst {

namespace {

struct Reader {
    const char* p;
    std::string err;

    void ws() {
        while (*p && isspace((unsigned char)*p)) ++p;
    }
    bool expect(char c) {
        ws();
        if (*p != c) {
            err = std::string("expected '") + c + "'";
            return false;
        }
        ++p;
        return true;
    }
    bool string(std::string* out) {
        ws();
        if (*p != '"') {
            err = "expected a string";
            return false;
        }
        ++p;
        out->clear();
        while (*p && *p != '"') {
            if (*p == '\\' && (p[1] == '"' || p[1] == '\\')) ++p;
            out->push_back(*p++);
        }
        if (*p != '"') {
            err = "unterminated string";
            return false;
        }
        ++p;
        return true;
    }
    bool integer(int64_t* out) {
        ws();
        char* end = nullptr;
        const long long v = strtoll(p, &end, 10);
        if (end == p) {
            err = "expected an integer";
            return false;
        }
        if (*end == '.' || *end == 'e' || *end == 'E') {
            err = "expected an integer";
            return false;
        }
        p = end;
        *out = (int64_t)v;
        return true;
    }
    // skip any value (used for keys the table does not know)
    bool skip() {
        ws();
        if (*p == '"') {
            std::string s;
            return string(&s);
        }
        if (*p == '{' || *p == '[') {
            const char open = *p, close = open == '{' ? '}' : ']';
            ++p;
            ws();
            if (*p == close) {
                ++p;
                return true;
            }
            for (;;) {
                if (open == '{') {
                    std::string k;
                    if (!string(&k) || !expect(':')) return false;
                }
                if (!skip()) return false;
                ws();
                if (*p == ',') {
                    ++p;
                    continue;
                }
                return expect(close);
            }
        }
        for (const char* lit : {"true", "false", "null"}) {
            const size_t L = strlen(lit);
            if (strncmp(p, lit, L) == 0) {
                p += L;
                return true;
            }
        }
        int64_t v;
        if (integer(&v)) return true;
        // a number with a fraction or exponent
        char* end = nullptr;
        strtod(p, &end);
        if (end == p) {
            err = "unexpected character";
            return false;
        }
        err.clear();
        p = end;
        return true;
    }
};

}  // namespace

bool TuneTable::parse(const char* json, uint32_t valid_variants, std::string* err) {
    Reader r{json, {}};
    std::vector<TuneEntry> out;
    auto fail = [&](const std::string& why) {
        if (err) *err = "autotune table: " + why;
        return false;
    };
    if (!r.expect('{')) return fail(r.err);
    r.ws();
    if (*r.p != '}') {
        for (;;) {
            std::string key;
            if (!r.string(&key) || !r.expect(':')) return fail(r.err);
            if (key == "entries") {
                if (!r.expect('[')) return fail(r.err);
                r.ws();
                if (*r.p == ']') {
                    ++r.p;
                } else {
                    for (;;) {
                        TuneEntry e{-1, -1, -1, -1, 8};
                        if (!r.expect('{')) return fail(r.err);
                        r.ws();
                        if (*r.p != '}') {
                            for (;;) {
                                std::string k;
                                if (!r.string(&k) || !r.expect(':')) return fail(r.err);
                                if (k == "mode") {
                                    std::string m;
                                    if (!r.string(&m)) return fail(r.err);
                                    if (m == "single") e.batched = 0;
                                    else if (m == "batched") e.batched = 1;
                                    else return fail("mode must be \"single\" or \"batched\"");
                                } else if (k == "dim" || k == "n_min" || k == "variant" || k == "lds_depth") {
                                    int64_t v;
                                    if (!r.integer(&v)) return fail(r.err);
                                    if (k == "dim") e.dim = (int)v;
                                    else if (k == "n_min") e.n_min = v;
                                    else if (k == "variant") e.variant = (int)v;
                                    else e.lds_depth = (v == 4 || v == 8 || v == 16) ? (int)v : -1;
                                } else if (!r.skip()) {
                                    return fail(r.err);
                                }
                                r.ws();
                                if (*r.p == ',') {
                                    ++r.p;
                                    continue;
                                }
                                if (!r.expect('}')) return fail(r.err);
                                break;
                            }
                        } else {
                            ++r.p;
                        }
                        if (e.batched < 0 || (e.dim != 2 && e.dim != 3) || e.n_min < 0 || e.variant < 0 ||
                            e.variant > 31 || !((valid_variants >> e.variant) & 1u) || e.lds_depth < 0)
                            return fail("every entry needs mode, dim in {2, 3}, n_min >= 0, a valid variant "
                                        "and lds_depth 4, 8 or 16 if given");
                        out.push_back(e);
                        r.ws();
                        if (*r.p == ',') {
                            ++r.p;
                            continue;
                        }
                        if (!r.expect(']')) return fail(r.err);
                        break;
                    }
                }
            } else if (!r.skip()) {
                return fail(r.err);
            }
            r.ws();
            if (*r.p == ',') {
                ++r.p;
                continue;
            }
            if (!r.expect('}')) return fail(r.err);
            break;
        }
    } else {
        ++r.p;
    }
    r.ws();
    if (*r.p) return fail("trailing characters");
    entries_ = out;
    return true;
}

const TuneEntry* TuneTable::pick(int batched, int dim, int64_t n) const {
    const TuneEntry* best = nullptr;
    for (const TuneEntry& e : entries_)
        if (e.batched == batched && e.dim == dim && e.n_min <= n && (!best || e.n_min > best->n_min)) best = &e;
    return best;
}

std::string TuneTable::dump() const {
    std::string s = "{\"entries\": [";
    char buf[160];
    for (size_t i = 0; i < entries_.size(); ++i) {
        const TuneEntry& e = entries_[i];
        snprintf(buf, sizeof(buf),
                 "%s{\"mode\": \"%s\", \"dim\": %d, \"n_min\": %lld, \"variant\": %d, \"lds_depth\": %d}",
                 i ? ", " : "", e.batched ? "batched" : "single", e.dim, (long long)e.n_min, e.variant, e.lds_depth);
        s += buf;
    }
    s += "]}";
    return s;
}

}  // namespace emst
