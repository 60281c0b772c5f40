// JSON tuning cache of the autotuner (host code only).
//
// The file holds one object:
//   {"format": "ecmg-tune-1", "device": "<name> <compute units> CUs",
//    "levels": {"<precision> <nx>x<ny>x<nz>": {"path": "tiled" | "persistent" | "gather",
//               "kz": K, "seg": S, "nwg": W, "us_default": D, "us_best": B}, ...,
//               "batch <precision>": {"path": "batch", "seg": S, "nwg": NPW, ...}}}
// keyed by the level's precision and elements per axis (the batched solve's
// entry: its segment length and nodes per workgroup).  The reader accepts any
// JSON whose top level has that shape (other keys ignored); the writer replaces
// the file through a temporary file and a rename, so a reader never sees half
// of it.
#include "ecmg_internal.h"

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

namespace ecmg {

namespace {

// A minimal JSON value: objects, strings and numbers are what the cache uses;
// arrays, booleans and null are parsed and skipped.
struct JVal {
    enum Kind { NUL, NUM, STR, OBJ, ARR, BOOL } kind = NUL;
    double num = 0.0;
    std::string str;
    std::vector<std::pair<std::string, JVal>> obj;
    std::vector<JVal> arr;
    const JVal *get(const std::string &k) const {
        for (auto &kv : obj)
            if (kv.first == k) return &kv.second;
        return nullptr;
    }
};

struct Parser {
    const std::string &s;
    size_t i = 0;
    std::string err;
    explicit Parser(const std::string &src) : s(src) {}
    void ws() {
        while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    }
    bool fail(const char *what) {
        if (err.empty()) err = std::string(what) + " at byte " + std::to_string(i);
        return false;
    }
    bool lit(const char *w) {
        const size_t n = std::strlen(w);
        if (s.compare(i, n, w) != 0) return fail("bad literal");
        i += n;
        return true;
    }
    bool string(std::string &out) {
        if (i >= s.size() || s[i] != '"') return fail("expected a string");
        ++i;
        out.clear();
        while (i < s.size() && s[i] != '"') {
            char c = s[i++];
            if (c == '\\') {
                if (i >= s.size()) return fail("bad escape");
                const char e = s[i++];
                if (e == 'n') c = '\n';
                else if (e == 't') c = '\t';
                else if (e == 'u') {                  // keys and values here are ASCII
                    if (i + 4 > s.size()) return fail("bad escape");
                    c = (char)std::strtol(s.substr(i, 4).c_str(), nullptr, 16);
                    i += 4;
                } else c = e;
            }
            out.push_back(c);
        }
        if (i >= s.size()) return fail("unterminated string");
        ++i;
        return true;
    }
    bool value(JVal &v, int depth) {
        if (depth > 32) return fail("nesting too deep");
        ws();
        if (i >= s.size()) return fail("unexpected end");
        const char c = s[i];
        if (c == '{') {
            v.kind = JVal::OBJ;
            ++i;
            ws();
            if (i < s.size() && s[i] == '}') { ++i; return true; }
            for (;;) {
                ws();
                std::string k;
                if (!string(k)) return false;
                ws();
                if (i >= s.size() || s[i] != ':') return fail("expected ':'");
                ++i;
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.obj.emplace_back(std::move(k), std::move(x));
                ws();
                if (i < s.size() && s[i] == ',') { ++i; continue; }
                if (i < s.size() && s[i] == '}') { ++i; return true; }
                return fail("expected ',' or '}'");
            }
        }
        if (c == '[') {
            v.kind = JVal::ARR;
            ++i;
            ws();
            if (i < s.size() && s[i] == ']') { ++i; return true; }
            for (;;) {
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.arr.push_back(std::move(x));
                ws();
                if (i < s.size() && s[i] == ',') { ++i; continue; }
                if (i < s.size() && s[i] == ']') { ++i; return true; }
                return fail("expected ',' or ']'");
            }
        }
        if (c == '"') {
            v.kind = JVal::STR;
            return string(v.str);
        }
        if (c == 't') { v.kind = JVal::BOOL; v.num = 1; return lit("true"); }
        if (c == 'f') { v.kind = JVal::BOOL; return lit("false"); }
        if (c == 'n') { v.kind = JVal::NUL; return lit("null"); }
        char *end = nullptr;
        v.num = std::strtod(s.c_str() + i, &end);
        if (end == s.c_str() + i) return fail("bad value");
        v.kind = JVal::NUM;
        i = (size_t)(end - s.c_str());
        return true;
    }
};

int num_field(const JVal &o, const char *k, double dflt) {
    const JVal *v = o.get(k);
    return (v && v->kind == JVal::NUM) ? (int)v->num : (int)dflt;
}
double dbl_field(const JVal &o, const char *k) {
    const JVal *v = o.get(k);
    return (v && v->kind == JVal::NUM) ? v->num : 0.0;
}

}  // namespace

std::string tune_key_batch(int precision) { return precision == ECMG_MIXED ? "batch mixed" : "batch fp64"; }

std::string tune_key(int precision, int nx, int ny, int nz) {
    char b[96];
    std::snprintf(b, sizeof b, "%s %dx%dx%d", precision == ECMG_MIXED ? "mixed" : "fp64", nx, ny, nz);
    return b;
}

int tune_cache_read(const std::string &path, std::string *device, std::map<std::string, TuneEntry> *out,
                    std::string *err) {
    std::ifstream f(path, std::ios::binary);
    if (!f) {
        *err = "cannot open tuning cache " + path;
        return ECMG_ENOENT;
    }
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string text = ss.str();
    Parser p(text);
    JVal root;
    if (!p.value(root, 0) || root.kind != JVal::OBJ) {
        *err = "tuning cache " + path + " is not a JSON object" + (p.err.empty() ? "" : ": " + p.err);
        return ECMG_EINVAL;
    }
    const JVal *fmt = root.get("format");
    if (!fmt || fmt->kind != JVal::STR || fmt->str != "ecmg-tune-1") {
        *err = "tuning cache " + path + ": format is not ecmg-tune-1";
        return ECMG_EINVAL;
    }
    if (device) {
        const JVal *d = root.get("device");
        *device = (d && d->kind == JVal::STR) ? d->str : std::string();
    }
    const JVal *lv = root.get("levels");
    if (lv && lv->kind == JVal::OBJ) {
        for (auto &kv : lv->obj) {
            if (kv.second.kind != JVal::OBJ) continue;
            const JVal &o = kv.second;
            const JVal *pth = o.get("path");
            TuneEntry e;
            const std::string pname = (pth && pth->kind == JVal::STR) ? pth->str : std::string();
            e.path = pname == "persistent" ? 1 : pname == "batch" ? 2 : pname == "gather" ? 3 : 0;
            e.kz = num_field(o, "kz", 0);
            e.seg = num_field(o, "seg", 0);
            e.nwg = num_field(o, "nwg", 0);
            e.us_default = dbl_field(o, "us_default");
            e.us_best = dbl_field(o, "us_best");
            if (e.path == 0 && e.kz < 1) continue;            // not a usable choice
            if (e.path == 1 && (e.seg < 1 || e.nwg < 1)) continue;
            if (e.path == 2 && (e.seg < 0 || e.nwg < 64)) continue;   // batch: seg 0 = by box size
            (*out)[kv.first] = e;
        }
    }
    return ECMG_OK;
}

int tune_cache_write(const std::string &path, const std::string &device,
                     const std::map<std::string, TuneEntry> &entries, std::string *err) {
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
        if (!f) {
            *err = "cannot write tuning cache " + tmp;
            return ECMG_EINVAL;
        }
        f << "{\n \"format\": \"ecmg-tune-1\",\n \"device\": \"" << device << "\",\n \"levels\": {";
        bool first = true;
        for (auto &kv : entries) {
            const TuneEntry &e = kv.second;
            char b[320];
            std::snprintf(b, sizeof b,
                          "%s\n  \"%s\": {\"path\": \"%s\", \"kz\": %d, \"seg\": %d, \"nwg\": %d, "
                          "\"us_default\": %.3f, \"us_best\": %.3f}",
                          first ? "" : ",", kv.first.c_str(),
                          e.path == 3 ? "gather" : e.path == 2 ? "batch" : e.path == 1 ? "persistent" : "tiled",
                          e.kz, e.seg,
                          e.nwg, e.us_default, e.us_best);
            f << b;
            first = false;
        }
        f << "\n }\n}\n";
        if (!f) {
            *err = "writing tuning cache " + tmp + " failed";
            return ECMG_EINVAL;
        }
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) {
        *err = "cannot replace tuning cache " + path;
        return ECMG_EINVAL;
    }
    return ECMG_OK;
}

}  // namespace ecmg
