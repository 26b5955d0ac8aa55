// Process-wide table of backprojection tilings read from the autotuner's JSON
// cache (host only).  The file maps keys
//   "<device name>|<storage>|na=<angles>|n=<columns>|N=<voxels>|rows=<rows>"
// to objects whose "choice" member is [slices_per_block, angles_per_block];
// other members (the tuner's timings) are skipped.  A small recursive-descent
// reader covers the JSON the tuner writes (objects, arrays, strings with
// escapes, numbers, true/false/null).
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "tp_internal.h"

namespace tp {
namespace {

struct TuneKey {
    std::string device;
    int storage, na, n, N;
    bool operator<(const TuneKey& o) const {
        return std::tie(device, storage, na, n, N) < std::tie(o.device, o.storage, o.na, o.n, o.N);
    }
};
struct TuneChoice {
    int rows, k, a;
};

std::mutex g_mu;
std::map<TuneKey, TuneChoice> g_table;

struct Reader {
    const char* p;
    const char* end;
    std::string err;

    void ws() {
        while (p < end && std::isspace(static_cast<unsigned char>(*p))) ++p;
    }
    bool fail(const char* what) {
        if (err.empty()) err = what;
        return false;
    }
    bool lit(const char* w) {
        const size_t m = std::strlen(w);
        if (static_cast<size_t>(end - p) < m || std::strncmp(p, w, m) != 0) return fail("bad literal");
        p += m;
        return true;
    }
    bool string(std::string* out) {
        ws();
        if (p >= end || *p != '"') return fail("expected a string");
        ++p;
        std::string s;
        while (p < end && *p != '"') {
            char c = *p++;
            if (c == '\\') {
                if (p >= end) return fail("unterminated escape");
                const char e = *p++;
                switch (e) {
                    case '"': s += '"'; break;
                    case '\\': s += '\\'; break;
                    case '/': s += '/'; break;
                    case 'b': s += '\b'; break;
                    case 'f': s += '\f'; break;
                    case 'n': s += '\n'; break;
                    case 'r': s += '\r'; break;
                    case 't': s += '\t'; break;
                    case 'u': {
                        if (end - p < 4) return fail("short \\u escape");
                        unsigned v = 0;
                        for (int i = 0; i < 4; ++i) {
                            const char h = *p++;
                            if (!std::isxdigit(static_cast<unsigned char>(h))) return fail("bad \\u escape");
                            v = v * 16 + static_cast<unsigned>(std::isdigit(static_cast<unsigned char>(h))
                                                                   ? h - '0'
                                                                   : (std::tolower(h) - 'a' + 10));
                        }
                        // keys are ASCII device names; keep other code points as UTF-8
                        if (v < 0x80) {
                            s += static_cast<char>(v);
                        } else if (v < 0x800) {
                            s += static_cast<char>(0xC0 | (v >> 6));
                            s += static_cast<char>(0x80 | (v & 0x3F));
                        } else {
                            s += static_cast<char>(0xE0 | (v >> 12));
                            s += static_cast<char>(0x80 | ((v >> 6) & 0x3F));
                            s += static_cast<char>(0x80 | (v & 0x3F));
                        }
                        break;
                    }
                    default: return fail("bad escape");
                }
            } else {
                s += c;
            }
        }
        if (p >= end) return fail("unterminated string");
        ++p;
        if (out) *out = s;
        return true;
    }
    bool number(double* out) {
        ws();
        const char* q = p;
        if (q < end && (*q == '-' || *q == '+')) ++q;
        while (q < end && (std::isdigit(static_cast<unsigned char>(*q)) || *q == '.' || *q == 'e' || *q == 'E' ||
                           *q == '-' || *q == '+'))
            ++q;
        if (q == p) return fail("expected a number");
        const std::string t(p, q);
        char* e = nullptr;
        const double v = std::strtod(t.c_str(), &e);
        if (e == nullptr || *e != '\0') return fail("bad number");
        p = q;
        if (out) *out = v;
        return true;
    }
    // Any value; numbers of a top-level array are collected into `nums`.
    bool value(std::vector<double>* nums, int depth) {
        if (depth > 64) return fail("nesting too deep");
        ws();
        if (p >= end) return fail("unexpected end");
        if (*p == '{') {
            ++p;
            ws();
            if (p < end && *p == '}') {
                ++p;
                return true;
            }
            for (;;) {
                if (!string(nullptr)) return false;
                ws();
                if (p >= end || *p != ':') return fail("expected ':'");
                ++p;
                if (!value(nullptr, depth + 1)) return false;
                ws();
                if (p < end && *p == ',') {
                    ++p;
                    continue;
                }
                if (p < end && *p == '}') {
                    ++p;
                    return true;
                }
                return fail("expected ',' or '}'");
            }
        }
        if (*p == '[') {
            ++p;
            ws();
            if (p < end && *p == ']') {
                ++p;
                return true;
            }
            for (;;) {
                ws();
                if (nums && p < end && (*p == '-' || std::isdigit(static_cast<unsigned char>(*p)))) {
                    double v;
                    if (!number(&v)) return false;
                    nums->push_back(v);
                } else if (!value(nullptr, depth + 1)) {
                    return false;
                }
                ws();
                if (p < end && *p == ',') {
                    ++p;
                    continue;
                }
                if (p < end && *p == ']') {
                    ++p;
                    return true;
                }
                return fail("expected ',' or ']'");
            }
        }
        if (*p == '"') return string(nullptr);
        if (*p == 't') return lit("true");
        if (*p == 'f') return lit("false");
        if (*p == 'n') return lit("null");
        return number(nullptr);
    }
};

bool parse_key(const std::string& key, TuneKey* k, int* rows) {
    // split from the right: the device name may hold any character
    std::vector<std::string> f;
    size_t e = key.size();
    for (int i = 0; i < 5; ++i) {
        const size_t b = key.rfind('|', e == 0 ? 0 : e - 1);
        if (b == std::string::npos || e == 0) return false;
        f.push_back(key.substr(b + 1, e - b - 1));
        e = b;
    }
    k->device = key.substr(0, e);
    const std::string& st = f[4];
    if (st == "f32") k->storage = TP_F32;
    else if (st == "f16") k->storage = TP_F16;
    else if (st == "bf16") k->storage = TP_BF16;
    else return false;
    auto field = [](const std::string& s, const char* name, int* out) {
        const size_t m = std::strlen(name);
        if (s.compare(0, m, name) != 0) return false;
        char* end = nullptr;
        const long v = std::strtol(s.c_str() + m, &end, 10);
        if (end == s.c_str() + m || *end != '\0' || v <= 0 || v > 1000000000L) return false;
        *out = static_cast<int>(v);
        return true;
    };
    return field(f[3], "na=", &k->na) && field(f[2], "n=", &k->n) && field(f[1], "N=", &k->N) &&
           field(f[0], "rows=", rows);
}

}  // namespace

int tune_table_load(const char* path, std::string* err) {
    if (path == nullptr) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table.clear();
        return 0;
    }
    FILE* f = std::fopen(path, "rb");
    if (!f) {
        *err = std::string("cannot open ") + path;
        return -1;
    }
    std::string text;
    char buf[65536];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) {
        text.append(buf, got);
        if (text.size() > (size_t{64} << 20)) {
            std::fclose(f);
            *err = "tuning table larger than 64 MiB";
            return -1;
        }
    }
    std::fclose(f);
    Reader r{text.data(), text.data() + text.size(), {}};
    std::map<TuneKey, TuneChoice> table;
    r.ws();
    if (r.p >= r.end || *r.p != '{') {
        *err = "tuning table is not a JSON object";
        return -1;
    }
    ++r.p;
    r.ws();
    bool empty = r.p < r.end && *r.p == '}';
    if (empty) ++r.p;
    while (!empty) {
        std::string key;
        if (!r.string(&key)) break;
        r.ws();
        if (r.p >= r.end || *r.p != ':') {
            r.fail("expected ':'");
            break;
        }
        ++r.p;
        // the entry: an object with "choice": [k, a]
        r.ws();
        if (r.p >= r.end || *r.p != '{') {
            r.fail("entry is not an object");
            break;
        }
        ++r.p;
        std::vector<double> choice;
        bool have_choice = false, ok = true;
        r.ws();
        if (r.p < r.end && *r.p == '}') {
            ++r.p;
        } else {
            for (;;) {
                std::string member;
                if (!r.string(&member)) { ok = false; break; }
                r.ws();
                if (r.p >= r.end || *r.p != ':') { ok = r.fail("expected ':'"); break; }
                ++r.p;
                if (member == "choice") {
                    choice.clear();
                    r.ws();
                    if (r.p >= r.end || *r.p != '[') { ok = r.fail("choice is not an array"); break; }
                    if (!r.value(&choice, 1)) { ok = false; break; }
                    have_choice = true;
                } else if (!r.value(nullptr, 1)) {
                    ok = false;
                    break;
                }
                r.ws();
                if (r.p < r.end && *r.p == ',') { ++r.p; continue; }
                if (r.p < r.end && *r.p == '}') { ++r.p; break; }
                ok = r.fail("expected ',' or '}'");
                break;
            }
        }
        if (!ok) break;
        TuneKey k;
        int rows = 0;
        if (!parse_key(key, &k, &rows)) {
            *err = "bad tuning key '" + key + "'";
            return -1;
        }
        if (!have_choice || choice.size() != 2) {
            *err = "entry '" + key + "' has no [slices, angles] choice";
            return -1;
        }
        const int kk = static_cast<int>(choice[0]), aa = static_cast<int>(choice[1]);
        if (kk != choice[0] || aa != choice[1] || !(kk == 1 || kk == 2 || kk == 4 || kk == 8 || kk == 16) ||
            !(aa == 8 || aa == 16 || aa == 32 || aa == 64) ||
            backproject_lds_bytes(static_cast<tp_dtype>(k.storage), kk, aa) > 160 * 1024) {
            *err = "entry '" + key + "' has an illegal tiling";
            return -1;
        }
        // several chunk heights of one shape: keep the tallest
        auto it = table.find(k);
        if (it == table.end() || rows > it->second.rows) table[k] = TuneChoice{rows, kk, aa};
        r.ws();
        if (r.p < r.end && *r.p == ',') {
            ++r.p;
            r.ws();
            continue;
        }
        if (r.p < r.end && *r.p == '}') {
            ++r.p;
            break;
        }
        r.fail("expected ',' or '}'");
        break;
    }
    if (!r.err.empty()) {
        char at[64];
        std::snprintf(at, sizeof at, " at byte %ld", static_cast<long>(r.p - text.data()));
        *err = "tuning table: " + r.err + at;
        return -1;
    }
    r.ws();
    if (r.p != r.end) {
        *err = "tuning table: trailing characters";
        return -1;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.swap(table);
    return static_cast<int>(g_table.size());
}

bool tune_table_lookup(const std::string& device, int storage, int na, int n, int N, int* k, int* a) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_table.empty()) return false;
    auto it = g_table.find(TuneKey{device, storage, na, n, N});
    if (it == g_table.end()) return false;
    *k = it->second.k;
    *a = it->second.a;
    return true;
}

bool tune_table_empty() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_table.empty();
}

}  // namespace tp
