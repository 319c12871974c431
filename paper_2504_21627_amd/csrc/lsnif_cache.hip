// Autotune cache: the launch parameters lsnif_autotune / lsnif_autotune_pairs
// chose, kept in a JSON file across processes, keyed by the device's
// architecture and the object's shape and precisions.  A context created with
// a cache path reads the file once; every object it builds whose key is there
// starts with the cached parameters (no timing), and every autotune call
// rewrites the file with its winners.  The parameters change speed only, never
// a result, so a stale or foreign entry costs time, not correctness.
//
// File layout (written by this unit; any JSON with the same shape is read):
//   {"lsnif_autotune_cache": 1,
//    "entries": {"<key>": {"sort_bits": 5, "pair_bits": 4, "hot_lds_bytes": 0,
//                          "walk_chunks": 1, "persistent": 0}, ...}}
// with key "<arch> V=<V> L=<L> F=<F> log2_T=<t> H=<H> width=<w> feat=<p> mlp=<p>".
#include <cerrno>
#include <cstdio>
#include <cstring>
#include <string>
#include <unistd.h>

#include "lsnif_internal.hpp"

namespace lsnif {

namespace {

const char *dtype_name(int d)
{
    switch (d) {
    case LSNIF_FP32: return "fp32";
    case LSNIF_FP16: return "fp16";
    case LSNIF_BF16: return "bf16";
    case LSNIF_FP8_E4M3: return "fp8";
    default: return "?";
    }
}

// A small JSON reader: objects, strings (with \" \\ \/ escapes), numbers, true /
// false / null; arrays are skipped.  Enough for this file's shape, strict on syntax.
struct Reader {
    const char *p, *end;
    std::string err;

    void ws()
    {
        while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
    }
    bool expect(char c)
    {
        ws();
        if (p < end && *p == c) {
            ++p;
            return true;
        }
        err = std::string("expected '") + c + "'";
        return false;
    }
    bool string(std::string &out)
    {
        out.clear();
        if (!expect('"')) return false;
        while (p < end && *p != '"') {
            char c = *p++;
            if (c == '\\') {
                if (p >= end) break;
                c = *p++;
                if (c != '"' && c != '\\' && c != '/') {
                    err = "unsupported string escape";
                    return false;
                }
            }
            out.push_back(c);
        }
        if (p >= end) {
            err = "unterminated string";
            return false;
        }
        ++p;
        return true;
    }
    bool number(double &v)
    {
        ws();
        char *q = nullptr;
        errno = 0;
        v = std::strtod(p, &q);
        if (q == p || q > end || errno) {
            err = "bad number";
            return false;
        }
        p = q;
        return true;
    }
    // Skips any value.
    bool skip()
    {
        ws();
        if (p >= end) {
            err = "unexpected end";
            return false;
        }
        if (*p == '"') {
            std::string s;
            return string(s);
        }
        if (*p == '{' || *p == '[') {
            const char close = *p == '{' ? '}' : ']';
            const bool obj = *p == '{';
            ++p;
            ws();
            if (p < end && *p == close) {
                ++p;
                return true;
            }
            for (;;) {
                if (obj) {
                    std::string k;
                    if (!string(k) || !expect(':')) return false;
                }
                if (!skip()) return false;
                ws();
                if (p < end && *p == ',') {
                    ++p;
                    continue;
                }
                return expect(close);
            }
        }
        for (const char *lit : {"true", "false", "null"}) {
            const size_t n = std::strlen(lit);
            if ((size_t)(end - p) >= n && std::strncmp(p, lit, n) == 0) {
                p += n;
                return true;
            }
        }
        double v;
        return number(v);
    }
    // Calls fn(key) for each member of an object; fn parses the value.
    template <typename Fn> bool members(Fn &&fn)
    {
        if (!expect('{')) return false;
        ws();
        if (p < end && *p == '}') {
            ++p;
            return true;
        }
        for (;;) {
            std::string k;
            if (!string(k) || !expect(':')) return false;
            if (!fn(k)) return false;
            ws();
            if (p < end && *p == ',') {
                ++p;
                continue;
            }
            return expect('}');
        }
    }
};

bool read_tuning(Reader &r, lsnif_tuning &t)
{
    int seen = 0;
    const bool ok = r.members([&](const std::string &k) -> bool {
        int32_t *dst = k == "sort_bits" ? &t.sort_bits
                       : k == "pair_bits" ? &t.pair_bits
                       : k == "hot_lds_bytes" ? &t.hot_lds_bytes
                       : k == "walk_chunks" ? &t.walk_chunks
                       : k == "persistent" ? &t.persistent
                                           : nullptr;
        if (!dst) return r.skip();
        double v;
        if (!r.number(v)) return false;
        if (v != (double)(int32_t)v) {
            r.err = "parameter " + k + " is not an integer";
            return false;
        }
        *dst = (int32_t)v;
        ++seen;
        return true;
    });
    if (ok && seen != 5) {
        r.err = "an entry needs sort_bits, pair_bits, hot_lds_bytes, walk_chunks and persistent";
        return false;
    }
    return ok;
}

}  // namespace

std::string device_arch(int device)
{
    if (device < 0) return "host";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

std::string cache_key(const lsnif_ctx *ctx, const Object &ob)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s V=%u L=%u F=%u log2_T=%u H=%u width=%d feat=%s mlp=%s", ctx->arch.c_str(),
                  ob.geom.V, ob.geom.L, ob.geom.F, ob.geom.log2_T, ob.geom.H, ob.width, dtype_name(ob.feat_dtype),
                  dtype_name(ob.mlp_dtype));
    return buf;
}

lsnif_status cache_load(lsnif_ctx *ctx)
{
    ctx->cache.clear();
    if (ctx->cache_path.empty()) return LSNIF_OK;
    FILE *f = std::fopen(ctx->cache_path.c_str(), "rb");
    if (!f) {
        if (errno == ENOENT) return LSNIF_OK;   // first use: the first autotune writes it
        return fail(LSNIF_E_INVALID, "autotune cache %s: %s", ctx->cache_path.c_str(), std::strerror(errno));
    }
    std::string text;
    char chunk[4096];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof chunk, f)) > 0) text.append(chunk, got);
    std::fclose(f);
    Reader r{text.data(), text.data() + text.size(), {}};
    std::map<std::string, lsnif_tuning> entries;
    int version = 0;
    const bool ok = r.members([&](const std::string &k) -> bool {
        if (k == "lsnif_autotune_cache") {
            double v;
            if (!r.number(v)) return false;
            version = (int)v;
            return true;
        }
        if (k != "entries") return r.skip();
        return r.members([&](const std::string &key) -> bool {
            lsnif_tuning t{};
            if (!read_tuning(r, t)) return false;
            entries[key] = t;
            return true;
        });
    });
    r.ws();
    if (!ok || r.p != r.end)
        return fail(LSNIF_E_INVALID, "autotune cache %s is not valid: %s at byte %ld", ctx->cache_path.c_str(),
                    ok ? "trailing characters" : r.err.c_str(), (long)(r.p - text.data()));
    if (version != 1)
        return fail(LSNIF_E_INVALID, "autotune cache %s: unknown version %d", ctx->cache_path.c_str(), version);
    for (const auto &kv : entries)
        if (lsnif_status st = check_tuning(&kv.second))
            return fail(st, "autotune cache %s, entry \"%s\": %s", ctx->cache_path.c_str(), kv.first.c_str(),
                        lsnif_last_error());
    ctx->cache = std::move(entries);
    return LSNIF_OK;
}

lsnif_status cache_save(lsnif_ctx *ctx)
{
    if (ctx->cache_path.empty()) return LSNIF_OK;
    std::string out = "{\"lsnif_autotune_cache\": 1,\n \"entries\": {";
    bool first = true;
    for (const auto &kv : ctx->cache) {
        char buf[192];
        std::snprintf(buf, sizeof buf,
                      "\": {\"sort_bits\": %d, \"pair_bits\": %d, \"hot_lds_bytes\": %d, \"walk_chunks\": %d, "
                      "\"persistent\": %d}",
                      kv.second.sort_bits, kv.second.pair_bits, kv.second.hot_lds_bytes, kv.second.walk_chunks,
                      kv.second.persistent);
        out += first ? "\n  \"" : ",\n  \"";
        for (char c : kv.first) {
            if (c == '"' || c == '\\') out.push_back('\\');
            out.push_back(c);
        }
        out += buf;
        first = false;
    }
    out += "\n }\n}\n";
    // write a sibling file, then rename it over the cache: readers never see half a file
    const std::string tmp = ctx->cache_path + ".tmp" + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(LSNIF_E_INVALID, "autotune cache %s: %s", tmp.c_str(), std::strerror(errno));
    const bool wrote = std::fwrite(out.data(), 1, out.size(), f) == out.size();
    if (std::fclose(f) != 0 || !wrote) {
        std::remove(tmp.c_str());
        return fail(LSNIF_E_INVALID, "autotune cache %s: write failed", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), ctx->cache_path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return fail(LSNIF_E_INVALID, "autotune cache %s: %s", ctx->cache_path.c_str(), std::strerror(errno));
    }
    return LSNIF_OK;
}

}  // namespace lsnif
