// Minimal JSON reader for process descriptions (objects, arrays, numbers,
// strings, true/false/null).  Host-only; errors are reported as strings.
#pragma once

#include <map>
#include <memory>
#include <string>
#include <vector>

namespace msx {

struct JValue {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    bool b = false;
    double num = 0.0;
    std::string str;
    std::vector<JValue> arr;
    std::vector<std::pair<std::string, JValue>> obj;

    const JValue* get(const std::string& key) const {
        if (kind != OBJ) return nullptr;
        for (const auto& kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
    bool has(const std::string& key) const { return get(key) != nullptr; }
    bool is_int() const { return kind == NUM && num == (double)(long long)num; }
};

// Parse `text`; on failure returns false and sets `err`.
bool parse_json(const std::string& text, JValue& out, std::string& err);

}  // namespace msx
