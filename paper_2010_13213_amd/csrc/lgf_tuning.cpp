// The MAC tuning table as JSON:
//
//   {"version": 2, "entries": {"<shape key>": {"choice": "pairs 16x8",
//     "candidates": ["pairs 16x8", "pairs 8x8", "pairs 16x16", "lattice"],
//     "ms": [42.7, 48.1, 45.6, 4.1]}, ...}}
//
// choice: the MAC method of convolutions of that shape, "pairs TYxTZ" (the
// block-pair kernel with TY x TZ target rows per workgroup) or "lattice"
// (the FFT over the block lattice); candidates / ms: every method timed and
// its milliseconds per MAC launch (both empty or absent for an entry written
// by hand).  The reader accepts any JSON of this form (whitespace, key
// order, extra keys in an entry) and rejects everything else with the byte
// offset of the problem.
#include <array>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "lgf_runtime.hpp"

namespace lgf {

namespace {

struct Reader {
    const std::string &s;
    size_t i = 0;

    [[noreturn]] void fail(const char *what) const {
        throw Failure(LGF_E_INVALID, "tuning JSON, byte " + std::to_string(i) + ": " + what);
    }
    void ws() {
        while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    }
    bool peek(char c) {
        ws();
        return i < s.size() && s[i] == c;
    }
    void expect(char c) {
        if (!peek(c)) {
            char m[32];
            std::snprintf(m, sizeof m, "expected '%c'", c);
            fail(m);
        }
        ++i;
    }
    std::string str() {
        expect('"');
        std::string out;
        while (i < s.size() && s[i] != '"') {
            if (s[i] == '\\') {
                if (++i >= s.size()) break;
                if (s[i] != '"' && s[i] != '\\' && s[i] != '/') fail("unsupported escape in a string");
            }
            out += s[i++];
        }
        if (i >= s.size()) fail("unterminated string");
        ++i;
        return out;
    }
    double num() {
        ws();
        const char *b = s.c_str() + i;
        char *e = nullptr;
        const double v = std::strtod(b, &e);
        if (e == b) fail("expected a number");
        i += (size_t)(e - b);
        return v;
    }
    int whole(int lo, int hi) {
        const double v = num();
        if (!(v >= lo && v <= hi) || v != std::floor(v)) fail("expected a whole number in range");
        return (int)v;
    }
    // skips any JSON value (for keys this reader does not use)
    void skip() {
        ws();
        if (i >= s.size()) fail("unexpected end");
        const char c = s[i];
        if (c == '"') {
            str();
        } else if (c == '{' || c == '[') {
            const char close = c == '{' ? '}' : ']';
            ++i;
            if (peek(close)) {
                ++i;
                return;
            }
            for (;;) {
                if (c == '{') {
                    str();
                    expect(':');
                }
                skip();
                if (peek(',')) {
                    ++i;
                    continue;
                }
                expect(close);
                return;
            }
        } else if (s.compare(i, 4, "true") == 0 || s.compare(i, 4, "null") == 0) {
            i += 4;
        } else if (s.compare(i, 5, "false") == 0) {
            i += 5;
        } else {
            num();
        }
    }
    // "{" (key ":" value ("," key ":" value)*)? "}", value read by f(key)
    template <typename F> void object(F &&f) {
        expect('{');
        if (peek('}')) {
            ++i;
            return;
        }
        for (;;) {
            const std::string k = str();
            expect(':');
            f(k);
            if (peek(',')) {
                ++i;
                continue;
            }
            expect('}');
            return;
        }
    }
    template <typename F> void array(F &&f) {
        expect('[');
        if (peek(']')) {
            ++i;
            return;
        }
        for (;;) {
            f();
            if (peek(',')) {
                ++i;
                continue;
            }
            expect(']');
            return;
        }
    }
};

void put_string(std::string &o, const std::string &k) {
    o += '"';
    for (char c : k) {
        if (c == '"' || c == '\\') o += '\\';
        o += c;
    }
    o += '"';
}

}  // namespace

bool parse_choice(const std::string &c, int &ty, int &tz) {
    if (c == "lattice") return true;
    int a = 0, b = 0, n = 0;
    if (std::sscanf(c.c_str(), "pairs %dx%d%n", &a, &b, &n) == 2 && n == (int)c.size() && a >= 1 && a <= 64 &&
        b >= 1 && b <= 64) {
        ty = a;
        tz = b;
        return false;
    }
    throw Failure(LGF_E_INVALID, "tuning choice '" + c + "' is neither 'lattice' nor 'pairs TYxTZ'");
}

std::string tuning_to_json(const std::map<std::string, TuneEntry> &table) {
    std::string o = "{\"version\": 2, \"entries\": {";
    bool first = true;
    char buf[64];
    for (const auto &kv : table) {
        o += first ? "\n  " : ",\n  ";
        first = false;
        put_string(o, kv.first);
        o += ": {\"choice\": ";
        put_string(o, kv.second.choice);
        o += ", \"candidates\": [";
        for (size_t c = 0; c < kv.second.cand.size(); ++c) {
            if (c) o += ", ";
            put_string(o, kv.second.cand[c]);
        }
        o += "], \"ms\": [";
        for (size_t c = 0; c < kv.second.ms.size(); ++c) {
            std::snprintf(buf, sizeof buf, "%s%.6g", c ? ", " : "", kv.second.ms[c]);
            o += buf;
        }
        o += "]}";
    }
    o += "\n}}\n";
    return o;
}

std::map<std::string, TuneEntry> tuning_from_json(const std::string &text) {
    Reader r{text};
    std::map<std::string, TuneEntry> out;
    bool have_entries = false;
    r.object([&](const std::string &k) {
        if (k == "version") {
            if (r.whole(2, 2) != 2) r.fail("unknown version");
        } else if (k == "entries") {
            have_entries = true;
            r.object([&](const std::string &key) {
                TuneEntry e;
                bool have_choice = false;
                r.object([&](const std::string &f) {
                    if (f == "choice") {
                        e.choice = r.str();
                        int ty, tz;
                        try {
                            parse_choice(e.choice, ty, tz);
                        } catch (const Failure &) {
                            r.fail("choice is neither \"lattice\" nor \"pairs TYxTZ\"");
                        }
                        have_choice = true;
                    } else if (f == "candidates") {
                        r.array([&] { e.cand.push_back(r.str()); });
                    } else if (f == "ms") {
                        r.array([&] { e.ms.push_back(r.num()); });
                    } else {
                        r.skip();
                    }
                });
                if (!have_choice) r.fail("an entry needs a choice");
                if (!e.ms.empty() && e.ms.size() != e.cand.size()) r.fail("ms and candidates differ in length");
                out[key] = e;
            });
        } else {
            r.skip();
        }
    });
    r.ws();
    if (r.i != text.size()) r.fail("trailing text");
    if (!have_entries) r.fail("no \"entries\" object");
    return out;
}

}  // namespace lgf
