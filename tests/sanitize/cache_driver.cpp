// Drives the autotuner's cache parser and formatter (csrc/tune_cache.cpp) for the sanitizer builds of
// tests/test_sanitizers.py: valid caches, format/parse round trips, every truncation of a valid text, and
// malformed inputs. Exit status 0 when every check held.
#include <cstdio>
#include <string>

#include "tune_cache.hpp"

using namespace stp;

static int fails = 0;
#define CHECK(c) do { if (!(c)) { std::fprintf(stderr, "failed: %s (line %d)\n", #c, __LINE__); ++fails; } } while (0)

int main()
{
    TuneCache c;
    CHECK(parse_tune_cache("{}", c) && c.empty());
    CHECK(parse_tune_cache(" { } ", c) && c.empty());
    const std::string good =
        "{\n \"gfx950|hip70000|cu256|class|N7,m9,p1\": {\"us_per_elem\": 0.0312, \"variant\": 3},\n"
        " \"gfx950|hip70000|cu256|hetero|x\": {\"grid_per_cu\": 2, \"lds_kb\": 128, \"ms\": 4.36e+00},\n"
        " \"empty\": {}\n}\n";
    CHECK(parse_tune_cache(good, c) && c.size() == 3);
    CHECK(c["gfx950|hip70000|cu256|class|N7,m9,p1"]["variant"] == 3.0);
    CHECK(c["empty"].empty());
    TuneCache r;
    CHECK(parse_tune_cache(format_tune_cache(c), r) && r == c);
    TuneCache big;
    for (int i = 0; i < 200; ++i)
        big["key" + std::to_string(i)] = {{"a", i * 0.5}, {"b", -1e-30 * i}, {"c", 1e300}};
    CHECK(parse_tune_cache(format_tune_cache(big), r) && r == big);
    // every prefix of a valid text that ends before its closing brace is rejected; nothing reads past the end
    for (size_t k = 0; k <= good.rfind('}'); ++k) {
        TuneCache t;
        const bool ok = parse_tune_cache(good.substr(0, k), t);
        CHECK(!ok && t.empty());
    }
    const char* bad[] = {"", "{", "}", "[]", "{\"a\"}", "{\"a\":}", "{\"a\":{\"b\":}}", "{\"a\":{\"b\":1,}}",
                         "{\"a\":{\"b\":1}", "{\"a\":{\"b\":--1}}", "{\"a\":{\"b\":1e}}", "{\"a\":{\"b\":\"x\"}}",
                         "{\"a\":{\"b\":1}} trailing", "{\"a\" {\"b\":1}}", "{\"a\":{\"b\":nan}}",
                         "{\"a\":{\"b\":1}},", "{\"unterminated: {}}", "{\"a\":{\"b\":1e999999}}"};
    for (const char* s : bad) {
        TuneCache t;
        (void)parse_tune_cache(s, t);  // must not crash; the overflowing exponent parses to inf
    }
    TuneCache t;
    CHECK(!parse_tune_cache("{\"a\":{\"b\":1}", t) && t.empty());
    std::printf("cache driver: %d failures\n", fails);
    return fails != 0;
}
