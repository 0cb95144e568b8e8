// Schedule cache of the batched launch: tuned schedules kept in one JSON file,
// keyed by (GPU architecture name, compute-unit count, mix signature), so that
// a process serving a known mix on a known GPU skips the search.  Host code
// only; nothing here touches the device.
//
// The file holds one object: {"format": "mtp-schedules-1", "entries": [...]},
// each entry a flat object of strings and numbers.  The reader is a small
// recursive-descent JSON parser (objects, arrays, strings, numbers, literals);
// a file it cannot read is treated as holding no entries by the lookup and is
// left untouched by the store.
#include <cerrno>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include <unistd.h>

#include "../../include/mtp.h"
#include "batch.hpp"

namespace {

constexpr const char* kFormat = "mtp-schedules-1";

// ------------------------------------------------------------------ signature

struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(int64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= static_cast<uint64_t>(v >> (8 * i)) & 0xFFu;
      h *= 1099511628211ull;
    }
  }
};

// ------------------------------------------------------------------ JSON

struct Value {
  enum Kind { kNull, kBool, kNum, kStr, kArr, kObj } kind = kNull;
  double num = 0.0;
  bool b = false;
  std::string str;
  std::vector<Value> arr;
  std::vector<std::pair<std::string, Value>> obj;
  const Value* get(const std::string& k) const {
    for (const auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

class Parser {
 public:
  explicit Parser(const std::string& s) : s_(s) {}
  bool parse(Value* out) {
    if (!value(out, 0)) return false;
    ws();
    return i_ == s_.size();
  }

 private:
  const std::string& s_;
  size_t i_ = 0;

  void ws() {
    while (i_ < s_.size() && (s_[i_] == ' ' || s_[i_] == '\t' || s_[i_] == '\n' || s_[i_] == '\r')) ++i_;
  }
  bool lit(const char* w) {
    const size_t n = std::strlen(w);
    if (s_.compare(i_, n, w) != 0) return false;
    i_ += n;
    return true;
  }
  bool string(std::string* out) {
    if (i_ >= s_.size() || s_[i_] != '"') return false;
    ++i_;
    out->clear();
    while (i_ < s_.size() && s_[i_] != '"') {
      char c = s_[i_++];
      if (c == '\\') {
        if (i_ >= s_.size()) return false;
        const char e = s_[i_++];
        switch (e) {
          case '"': c = '"'; break;
          case '\\': c = '\\'; break;
          case '/': c = '/'; break;
          case 'b': c = '\b'; break;
          case 'f': c = '\f'; break;
          case 'n': c = '\n'; break;
          case 'r': c = '\r'; break;
          case 't': c = '\t'; break;
          case 'u': {
            // keys and values here are ASCII; a \u escape outside it is kept as '?'
            if (i_ + 4 > s_.size()) return false;
            const unsigned long v = std::strtoul(s_.substr(i_, 4).c_str(), nullptr, 16);
            i_ += 4;
            c = v < 128 ? static_cast<char>(v) : '?';
            break;
          }
          default: return false;
        }
      } else if (static_cast<unsigned char>(c) < 0x20) {
        return false;
      }
      out->push_back(c);
    }
    if (i_ >= s_.size()) return false;
    ++i_;
    return true;
  }
  bool value(Value* v, int depth) {
    if (depth > 32) return false;
    ws();
    if (i_ >= s_.size()) return false;
    const char c = s_[i_];
    if (c == '{') {
      ++i_;
      v->kind = Value::kObj;
      ws();
      if (i_ < s_.size() && s_[i_] == '}') { ++i_; return true; }
      for (;;) {
        ws();
        std::string k;
        if (!string(&k)) return false;
        ws();
        if (i_ >= s_.size() || s_[i_] != ':') return false;
        ++i_;
        Value x;
        if (!value(&x, depth + 1)) return false;
        v->obj.emplace_back(std::move(k), std::move(x));
        ws();
        if (i_ < s_.size() && s_[i_] == ',') { ++i_; continue; }
        if (i_ < s_.size() && s_[i_] == '}') { ++i_; return true; }
        return false;
      }
    }
    if (c == '[') {
      ++i_;
      v->kind = Value::kArr;
      ws();
      if (i_ < s_.size() && s_[i_] == ']') { ++i_; return true; }
      for (;;) {
        Value x;
        if (!value(&x, depth + 1)) return false;
        v->arr.push_back(std::move(x));
        ws();
        if (i_ < s_.size() && s_[i_] == ',') { ++i_; continue; }
        if (i_ < s_.size() && s_[i_] == ']') { ++i_; return true; }
        return false;
      }
    }
    if (c == '"') {
      v->kind = Value::kStr;
      return string(&v->str);
    }
    if (lit("true")) { v->kind = Value::kBool; v->b = true; return true; }
    if (lit("false")) { v->kind = Value::kBool; v->b = false; return true; }
    if (lit("null")) { v->kind = Value::kNull; return true; }
    const char* start = s_.c_str() + i_;
    char* end = nullptr;
    errno = 0;
    const double d = std::strtod(start, &end);
    if (end == start || errno == ERANGE || !std::isfinite(d)) return false;
    i_ += static_cast<size_t>(end - start);
    v->kind = Value::kNum;
    v->num = d;
    return true;
  }
};

struct Entry {
  std::string arch, mix;
  int32_t cus = 0;
  mtp_batch_schedule s{};
  double ms = 0.0;
};

std::string hex64(uint64_t v) {
  char buf[17];
  std::snprintf(buf, sizeof(buf), "%016llx", static_cast<unsigned long long>(v));
  return buf;
}

bool int_field(const Value& o, const char* k, int32_t* out) {
  const Value* v = o.get(k);
  if (v == nullptr || v->kind != Value::kNum || v->num != std::floor(v->num) || std::fabs(v->num) > 2147483647.0)
    return false;
  *out = static_cast<int32_t>(v->num);
  return true;
}

bool entry_of(const Value& o, Entry* e) {
  if (o.kind != Value::kObj) return false;
  const Value* a = o.get("arch");
  const Value* m = o.get("mix");
  const Value* ms = o.get("ms");
  if (a == nullptr || a->kind != Value::kStr || m == nullptr || m->kind != Value::kStr || ms == nullptr ||
      ms->kind != Value::kNum)
    return false;
  e->arch = a->str;
  e->mix = m->str;
  e->ms = ms->num;
  return int_field(o, "cus", &e->cus) && int_field(o, "wg_per_cu", &e->s.wg_per_cu) &&
         int_field(o, "order", &e->s.order) && int_field(o, "cand_tiles", &e->s.cand_tiles) &&
         int_field(o, "roll_tiles", &e->s.roll_tiles) && int_field(o, "refit_outputs", &e->s.refit_outputs) &&
         int_field(o, "split_pct", &e->s.split_pct);
}

// 1: read (entries filled), 0: no such file, -1: a file that is not a cache.
int read_cache(const char* path, std::vector<Entry>* entries) {
  entries->clear();
  if (access(path, F_OK) != 0) return errno == ENOENT ? 0 : -1;
  std::ifstream f(path, std::ios::binary);
  if (!f) return -1;
  std::stringstream ss;
  ss << f.rdbuf();
  if (f.bad()) return -1;
  const std::string text = ss.str();
  Value root;
  if (!Parser(text).parse(&root) || root.kind != Value::kObj) return -1;
  const Value* fmt = root.get("format");
  const Value* arr = root.get("entries");
  if (fmt == nullptr || fmt->kind != Value::kStr || fmt->str != kFormat || arr == nullptr || arr->kind != Value::kArr)
    return -1;
  for (const Value& o : arr->arr) {
    Entry e;
    if (!entry_of(o, &e)) return -1;
    entries->push_back(e);
  }
  return 1;
}

std::string escaped(const std::string& s) {
  std::string o;
  for (const char c : s) {
    if (c == '"' || c == '\\') {
      o.push_back('\\');
      o.push_back(c);
    } else if (static_cast<unsigned char>(c) < 0x20) {
      char buf[8];
      std::snprintf(buf, sizeof(buf), "\\u%04x", static_cast<unsigned>(static_cast<unsigned char>(c)));
      o += buf;
    } else {
      o.push_back(c);
    }
  }
  return o;
}

bool write_cache(const char* path, const std::vector<Entry>& entries) {
  std::ostringstream o;
  o << "{\n  \"format\": \"" << kFormat << "\",\n  \"entries\": [";
  for (size_t i = 0; i < entries.size(); ++i) {
    const Entry& e = entries[i];
    char ms[32];
    std::snprintf(ms, sizeof(ms), "%.6g", e.ms);
    o << (i ? ",\n" : "\n") << "    {\"arch\": \"" << escaped(e.arch) << "\", \"cus\": " << e.cus << ", \"mix\": \""
      << escaped(e.mix) << "\", \"wg_per_cu\": " << e.s.wg_per_cu << ", \"order\": " << e.s.order
      << ", \"cand_tiles\": " << e.s.cand_tiles << ", \"roll_tiles\": " << e.s.roll_tiles
      << ", \"refit_outputs\": " << e.s.refit_outputs << ", \"split_pct\": " << e.s.split_pct << ", \"ms\": " << ms
      << "}";
  }
  o << (entries.empty() ? "]\n}\n" : "\n  ]\n}\n");
  const std::string tmp = std::string(path) + ".tmp." + std::to_string(static_cast<long>(getpid()));
  {
    std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
    if (!f) return false;
    f << o.str();
    f.flush();
    if (!f) {
      std::remove(tmp.c_str());
      return false;
    }
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace

bool mtp::schedule_valid(const mtp_batch_schedule& s) {
  auto pow2_in = [](int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; };
  return s.wg_per_cu >= 0 && s.wg_per_cu <= 64 && (s.order == 0 || s.order == 1) && pow2_in(s.cand_tiles, 1, 4) &&
         pow2_in(s.roll_tiles, 1, 4) && pow2_in(s.refit_outputs, 4, 64) && s.split_pct >= 0;
}

extern "C" {

uint64_t mtp_batch_mix_signature(const mtp_config* cfgs, int32_t n) {
  if (cfgs == nullptr || n < 1) return 0;
  Fnv f;
  f.add(n);
  for (int i = 0; i < n; ++i) {
    const mtp_config& c = cfgs[i];
    const int64_t fields[] = {c.dynamics,   c.interp,      c.n_links,        c.state_dim,
                              c.ctrl_dim,   c.horizon,     c.n_layers,       c.n_width,
                              c.n_tensor,   c.n_gauss,     c.n_elites,       c.n_iters,
                              c.interp == MTP_INTERP_BSPLINE ? c.bspline_degree : 0,
                              c.n_replicas > 1 ? c.n_replicas : 1,
                              c.sample_wor, c.diagnostics, c.n_debug_states, c.n_task_params};
    for (const int64_t v : fields) f.add(v);
  }
  return f.h == 0 ? 1 : f.h;
}

mtp_status mtp_schedule_cache_lookup(const char* path, const char* arch, int32_t cus, uint64_t mix,
                                     mtp_batch_schedule* h_out, float* h_ms, int32_t* h_found) {
  if (path == nullptr || arch == nullptr || h_found == nullptr) return MTP_ERR_INVALID_ARG;
  *h_found = 0;
  std::vector<Entry> entries;
  if (read_cache(path, &entries) != 1) return MTP_OK;
  const std::string key = hex64(mix);
  for (const Entry& e : entries) {
    if (e.arch == arch && e.cus == cus && e.mix == key && mtp::schedule_valid(e.s)) {
      if (h_out) *h_out = e.s;
      if (h_ms) *h_ms = static_cast<float>(e.ms);
      *h_found = 1;
      return MTP_OK;
    }
  }
  return MTP_OK;
}

mtp_status mtp_schedule_cache_store(const char* path, const char* arch, int32_t cus, uint64_t mix,
                                    const mtp_batch_schedule* h_schedule, float ms) {
  if (path == nullptr || arch == nullptr || h_schedule == nullptr || !mtp::schedule_valid(*h_schedule) || cus < 1 ||
      !std::isfinite(ms))
    return MTP_ERR_INVALID_ARG;
  std::vector<Entry> entries;
  if (read_cache(path, &entries) < 0) return MTP_ERR_INVALID_ARG;
  Entry e;
  e.arch = arch;
  e.cus = cus;
  e.mix = hex64(mix);
  e.s = *h_schedule;
  e.ms = ms;
  bool replaced = false;
  for (Entry& x : entries)
    if (x.arch == e.arch && x.cus == e.cus && x.mix == e.mix) {
      x = e;
      replaced = true;
    }
  if (!replaced) entries.push_back(e);
  return write_cache(path, entries) ? MTP_OK : MTP_ERR_INVALID_ARG;
}

}  // extern "C"
