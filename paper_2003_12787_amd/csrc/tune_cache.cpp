// tune_cache.cpp -- parse and format the autotuner's JSON cache (host only; see tune_cache.hpp).
#include "tune_cache.hpp"

#include <cstdio>
#include <cstdlib>

namespace stp {

namespace {

void skip_ws(const std::string& s, size_t& i)
{
    while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i;
}

bool read_string(const std::string& s, size_t& i, std::string& out)
{
    skip_ws(s, i);
    if (i >= s.size() || s[i] != '"') return false;
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) return false;
    out = s.substr(i + 1, j - i - 1);
    i = j + 1;
    return true;
}

bool expect(const std::string& s, size_t& i, char c)
{
    skip_ws(s, i);
    if (i >= s.size() || s[i] != c) return false;
    ++i;
    return true;
}

// A number at s[i..]: strtod on a bounded copy, so the scan never runs past the text.
bool read_number(const std::string& s, size_t& i, double& v)
{
    skip_ws(s, i);
    size_t j = i;
    while (j < s.size() && j - i < 64 &&
           (s[j] == '-' || s[j] == '+' || s[j] == '.' || s[j] == 'e' || s[j] == 'E' || (s[j] >= '0' && s[j] <= '9')))
        ++j;
    if (j == i) return false;
    const std::string tok = s.substr(i, j - i);
    char* end = nullptr;
    v = std::strtod(tok.c_str(), &end);
    if (end != tok.c_str() + tok.size()) return false;
    i = j;
    return true;
}

bool parse(const std::string& s, TuneCache& c)
{
    size_t i = 0;
    if (!expect(s, i, '{')) return false;
    skip_ws(s, i);
    if (i < s.size() && s[i] == '}') return true;
    for (;;) {
        std::string key;
        if (!read_string(s, i, key) || !expect(s, i, ':') || !expect(s, i, '{')) return false;
        TuneEntry e;
        skip_ws(s, i);
        if (i < s.size() && s[i] == '}') {
            ++i;
        } else {
            for (;;) {
                std::string name;
                double v;
                if (!read_string(s, i, name) || !expect(s, i, ':') || !read_number(s, i, v)) return false;
                e[name] = v;
                skip_ws(s, i);
                if (i < s.size() && s[i] == ',') {
                    ++i;
                    continue;
                }
                if (!expect(s, i, '}')) return false;
                break;
            }
        }
        c[key] = e;
        skip_ws(s, i);
        if (i < s.size() && s[i] == ',') {
            ++i;
            continue;
        }
        return expect(s, i, '}');
    }
}

}  // namespace

bool parse_tune_cache(const std::string& text, TuneCache& out)
{
    TuneCache c;
    if (!parse(text, c)) {
        out.clear();
        return false;
    }
    out.swap(c);
    return true;
}

std::string format_tune_cache(const TuneCache& c)
{
    std::string s = "{\n";
    size_t n = 0;
    char num[64];
    for (auto& kv : c) {
        s += " \"" + kv.first + "\": {";
        size_t m = 0;
        for (auto& e : kv.second) {
            std::snprintf(num, sizeof num, "%.17g", e.second);  // round-trips exactly
            s += (m++ ? ", \"" : "\"") + e.first + "\": " + num;
        }
        s += ++n < c.size() ? "},\n" : "}\n";
    }
    return s + "}\n";
}

}  // namespace stp
