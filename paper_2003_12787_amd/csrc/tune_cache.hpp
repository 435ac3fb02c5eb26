// tune_cache.hpp -- the autotuner's cache format (host only): one JSON object mapping a key to an object of
// numbers. Only that shape is written or read; anything else parses as an empty cache.
#pragma once
#include <map>
#include <string>

namespace stp {

using TuneEntry = std::map<std::string, double>;
using TuneCache = std::map<std::string, TuneEntry>;

// Parse `text`; returns false (and leaves `out` empty) for anything that is not exactly that shape.
bool parse_tune_cache(const std::string& text, TuneCache& out);

// The cache as JSON text (keys and names are written verbatim and must not contain '"' or '\').
std::string format_tune_cache(const TuneCache& c);

}  // namespace stp
