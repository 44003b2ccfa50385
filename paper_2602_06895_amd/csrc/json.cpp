#include "json.h"

#include <cctype>
#include <cstdlib>

namespace msx {
namespace {

struct Reader {
    const std::string& s;
    size_t i = 0;
    std::string err;
    int depth = 0;

    explicit Reader(const std::string& t) : s(t) {}

    void ws() {
        while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    }
    bool fail(const std::string& m) {
        if (err.empty()) err = m + " at offset " + std::to_string(i);
        return false;
    }
    bool lit(const char* w) {
        size_t n = 0;
        while (w[n]) ++n;
        if (s.compare(i, n, w) != 0) return fail(std::string("expected ") + w);
        i += n;
        return true;
    }
    bool string(std::string& out) {
        if (i >= s.size() || s[i] != '"') return fail("expected string");
        ++i;
        out.clear();
        while (i < s.size() && s[i] != '"') {
            char c = s[i++];
            if (c == '\\') {
                if (i >= s.size()) return fail("bad escape");
                char e = s[i++];
                switch (e) {
                    case '"': out += '"'; break;
                    case '\\': out += '\\'; break;
                    case '/': out += '/'; break;
                    case 'n': out += '\n'; break;
                    case 't': out += '\t'; break;
                    case 'r': out += '\r'; break;
                    case 'b': out += '\b'; break;
                    case 'f': out += '\f'; break;
                    default: return fail("unsupported escape");
                }
            } else {
                out += c;
            }
        }
        if (i >= s.size()) return fail("unterminated string");
        ++i;
        return true;
    }
    bool value(JValue& v) {
        if (++depth > 64) return fail("nesting too deep");
        ws();
        if (i >= s.size()) return fail("unexpected end");
        char c = s[i];
        bool ok;
        if (c == '{') {
            v.kind = JValue::OBJ;
            ++i;
            ws();
            ok = true;
            if (i < s.size() && s[i] == '}') {
                ++i;
            } else {
                while (true) {
                    ws();
                    std::string key;
                    if (!string(key)) { ok = false; break; }
                    ws();
                    if (i >= s.size() || s[i] != ':') { ok = fail("expected ':'"); break; }
                    ++i;
                    JValue child;
                    if (!value(child)) { ok = false; break; }
                    v.obj.emplace_back(key, std::move(child));
                    ws();
                    if (i < s.size() && s[i] == ',') { ++i; continue; }
                    if (i < s.size() && s[i] == '}') { ++i; break; }
                    ok = fail("expected ',' or '}'");
                    break;
                }
            }
        } else if (c == '[') {
            v.kind = JValue::ARR;
            ++i;
            ws();
            ok = true;
            if (i < s.size() && s[i] == ']') {
                ++i;
            } else {
                while (true) {
                    JValue child;
                    if (!value(child)) { ok = false; break; }
                    v.arr.push_back(std::move(child));
                    ws();
                    if (i < s.size() && s[i] == ',') { ++i; continue; }
                    if (i < s.size() && s[i] == ']') { ++i; break; }
                    ok = fail("expected ',' or ']'");
                    break;
                }
            }
        } else if (c == '"') {
            v.kind = JValue::STR;
            ok = string(v.str);
        } else if (c == 't') {
            v.kind = JValue::BOOL;
            v.b = true;
            ok = lit("true");
        } else if (c == 'f') {
            v.kind = JValue::BOOL;
            v.b = false;
            ok = lit("false");
        } else if (c == 'n') {
            v.kind = JValue::NUL;
            ok = lit("null");
        } else {
            const char* b = s.c_str() + i;
            char* e = nullptr;
            v.kind = JValue::NUM;
            v.num = std::strtod(b, &e);
            if (e == b) {
                ok = fail("unexpected character");
            } else {
                i += (size_t)(e - b);
                ok = true;
            }
        }
        --depth;
        return ok;
    }
};

}  // namespace

bool parse_json(const std::string& text, JValue& out, std::string& err) {
    Reader r(text);
    if (!r.value(out)) {
        err = r.err;
        return false;
    }
    r.ws();
    if (r.i != text.size()) {
        err = "trailing characters at offset " + std::to_string(r.i);
        return false;
    }
    return true;
}

}  // namespace msx
