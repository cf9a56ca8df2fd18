// Autotuner for batched plans (rel_autotune, rel_autotune_lookup).
//
// Batch execution is the paper's answer to many small queries that leave a
// GPU underused (Section 5, future work); the knobs that decide how a batch
// instance uses the chip are the hash-table load factor, the fan-out of an
// instance over the persistent workgroups (fact tiles per work item), the
// block shape (resident workgroups per CU, and the LDS group table that sets
// how many fit) and the copies of the global group table. For each sample
// plan this file times every candidate record on the GPU as a one-plan
// batch, checks that every candidate returns the same groups (a difference
// is a race), keeps the fastest, and stores it in a JSON file keyed by
// (GPU architecture, operation, size bucket). A bucket is the magnitude, in
// steps of 4x, of the fact rows, the largest dim and the group bound: plans
// of one bucket share the trade-offs the knobs make.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"
#include "rel.h"

namespace rel {
namespace {

// ------------------------------------------------------------ JSON values
//
// The subset the cache needs: objects, strings, numbers, booleans, null and
// arrays; objects keep their keys sorted.

struct Json {
  enum Kind { kNull, kBool, kNum, kStr, kArr, kObj } kind = kNull;
  double num = 0;
  bool b = false;
  std::string str;
  std::vector<Json> arr;
  std::map<std::string, Json> obj;
};

struct Parser {
  const std::string& s;
  size_t i = 0;
  bool ok = true;
  explicit Parser(const std::string& text) : s(text) {}

  void ws() {
    while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\t' || s[i] == '\r')) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  std::string string() {
    std::string out;
    if (!eat('"')) {
      ok = false;
      return out;
    }
    while (i < s.size() && s[i] != '"') {
      char c = s[i++];
      if (c == '\\' && i < s.size()) {
        const char e = s[i++];
        if (e == 'n') c = '\n';
        else if (e == 't') c = '\t';
        else if (e == 'u') {  // \uXXXX: only ASCII is ever written here
          c = static_cast<char>(std::strtol(s.substr(i, 4).c_str(), nullptr, 16));
          i += 4;
        } else {
          c = e;
        }
      }
      out.push_back(c);
    }
    if (i >= s.size()) ok = false;
    ++i;
    return out;
  }
  Json value() {
    Json v;
    ws();
    if (i >= s.size()) {
      ok = false;
      return v;
    }
    const char c = s[i];
    if (c == '{') {
      ++i;
      v.kind = Json::kObj;
      if (eat('}')) return v;
      do {
        std::string k = string();
        if (!eat(':')) ok = false;
        v.obj[k] = value();
      } while (ok && eat(','));
      if (!eat('}')) ok = false;
    } else if (c == '[') {
      ++i;
      v.kind = Json::kArr;
      if (eat(']')) return v;
      do v.arr.push_back(value());
      while (ok && eat(','));
      if (!eat(']')) ok = false;
    } else if (c == '"') {
      v.kind = Json::kStr;
      v.str = string();
    } else if (s.compare(i, 4, "true") == 0) {
      v.kind = Json::kBool;
      v.b = true;
      i += 4;
    } else if (s.compare(i, 5, "false") == 0) {
      v.kind = Json::kBool;
      i += 5;
    } else if (s.compare(i, 4, "null") == 0) {
      i += 4;
    } else {
      char* end = nullptr;
      v.num = std::strtod(s.c_str() + i, &end);
      if (end == s.c_str() + i) ok = false;
      v.kind = Json::kNum;
      i = static_cast<size_t>(end - s.c_str());
    }
    return v;
  }
};

void dump(const Json& v, std::string& out, int indent) {
  const std::string pad(static_cast<size_t>(indent), ' ');
  switch (v.kind) {
    case Json::kNull: out += "null"; break;
    case Json::kBool: out += v.b ? "true" : "false"; break;
    case Json::kNum: {
      char buf[64];
      if (v.num == std::floor(v.num) && std::fabs(v.num) < 1e15)
        std::snprintf(buf, sizeof buf, "%lld", static_cast<long long>(v.num));
      else
        std::snprintf(buf, sizeof buf, "%.17g", v.num);
      out += buf;
      break;
    }
    case Json::kStr: {
      out.push_back('"');
      for (char c : v.str) {
        if (c == '"' || c == '\\') out.push_back('\\');
        out.push_back(c);
      }
      out.push_back('"');
      break;
    }
    case Json::kArr: {
      out += "[";
      for (size_t k = 0; k < v.arr.size(); ++k) {
        if (k) out += ", ";
        dump(v.arr[k], out, indent);
      }
      out += "]";
      break;
    }
    case Json::kObj: {
      if (v.obj.empty()) {
        out += "{}";
        break;
      }
      out += "{\n";
      size_t k = 0;
      for (const auto& kv : v.obj) {
        out += pad + " ";
        Json key;
        key.kind = Json::kStr;
        key.str = kv.first;
        dump(key, out, indent + 1);
        out += ": ";
        dump(kv.second, out, indent + 1);
        out += ++k < v.obj.size() ? ",\n" : "\n";
      }
      out += pad + "}";
      break;
    }
  }
}

Json number(double x) {
  Json v;
  v.kind = Json::kNum;
  v.num = x;
  return v;
}

bool read_cache(const char* path, Json& root) {
  root = Json();
  root.kind = Json::kObj;
  std::ifstream f(path);
  if (!f) return true;  // no cache yet
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  Parser p(text);
  Json v = p.value();
  if (!p.ok || v.kind != Json::kObj) return false;
  root = v;
  return true;
}

bool write_cache(const char* path, const Json& root) {
  std::string out;
  dump(root, out, 0);
  out += "\n";
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return false;
    f << out;
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

// ---------------------------------------------------------- buckets, keys

int magnitude(int64_t x) {
  if (x <= 1) return 0;
  return static_cast<int>(std::ceil(std::log2(static_cast<double>(x))));
}

std::string bucket_of(const rel_pipeline_desc& d) {
  int64_t dim = 0;
  for (int i = 0; i < d.n_dims; ++i) dim = std::max(dim, d.dims[i].key.len);
  auto step = [](int64_t x) { return 2 * (magnitude(x) / 2); };
  char buf[64];
  std::snprintf(buf, sizeof buf, "f%d-d%d-g%d", step(d.fact[0].len), step(dim),
                step(d.max_groups));
  return buf;
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "none";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

constexpr const char* kOp = "pipeline_batch";

std::string cache_key(const std::string& arch, const rel_pipeline_desc& d) {
  return arch + "/" + kOp + "/" + bucket_of(d);
}

// ------------------------------------------------------------- candidates

// Fields of rel_tuning a record may set (the names the JSON uses).
struct Field {
  const char* name;
  bool is_float;
};
constexpr Field kFields[] = {{"load_factor", true}, {"lds_slots", false}, {"replicas", false},
                             {"chunk_tiles", false}, {"grid", false},     {"fanout", false},
                             {"dim_lds_bytes", false}};

double get_field(const rel_tuning& t, const char* name) {
  if (!std::strcmp(name, "load_factor")) return t.load_factor;
  if (!std::strcmp(name, "lds_slots")) return t.lds_slots;
  if (!std::strcmp(name, "replicas")) return t.replicas;
  if (!std::strcmp(name, "chunk_tiles")) return t.chunk_tiles;
  if (!std::strcmp(name, "grid")) return t.grid;
  if (!std::strcmp(name, "fanout")) return t.fanout;
  return t.dim_lds_bytes;
}

void set_field(rel_tuning& t, const std::string& name, double v) {
  if (name == "load_factor") t.load_factor = static_cast<float>(v);
  else if (name == "lds_slots") t.lds_slots = static_cast<int32_t>(v);
  else if (name == "replicas") t.replicas = static_cast<int32_t>(v);
  else if (name == "chunk_tiles") t.chunk_tiles = static_cast<int32_t>(v);
  else if (name == "grid") t.grid = static_cast<int32_t>(v);
  else if (name == "fanout") t.fanout = static_cast<int32_t>(v);
  else if (name == "dim_lds_bytes") t.dim_lds_bytes = static_cast<int32_t>(v);
}

// The record's non-default fields as a JSON object (and its text, which
// names the candidate in the record).
Json record_of(const rel_tuning& t) {
  Json o;
  o.kind = Json::kObj;
  for (const Field& f : kFields) {
    const double v = get_field(t, f.name);
    if (v != 0) o.obj[f.name] = number(f.is_float ? std::round(v * 1e6) / 1e6 : v);
  }
  return o;
}

std::string compact(const Json& o) {
  std::string s = "{";
  size_t k = 0;
  for (const auto& kv : o.obj) {
    std::string v;
    dump(kv.second, v, 0);
    s += "\"" + kv.first + "\": " + v + (++k < o.obj.size() ? ", " : "");
  }
  return s + "}";
}

// Load factor, work split (fact tiles per work item of a batch instance),
// block shape (resident workgroups: the LDS group table's size, or a fixed
// number of workgroups per CU), global group-table copies, and the fan-out
// of a batched plan's spilled-row records (their partitions, or none).
std::vector<rel_tuning> candidates(int cu) {
  std::vector<rel_tuning> c;
  auto add = [&](std::initializer_list<std::pair<const char*, double>> fields) {
    rel_tuning t;
    std::memset(&t, 0, sizeof t);
    for (const auto& f : fields) set_field(t, f.first, f.second);
    c.push_back(t);
  };
  add({});
  add({{"replicas", 1}});
  add({{"replicas", 8}});
  add({{"replicas", 32}});
  add({{"replicas", 64}});
  add({{"lds_slots", -1}, {"replicas", 32}});
  add({{"load_factor", 0.3}});
  add({{"load_factor", 0.3}, {"replicas", 32}});
  add({{"lds_slots", 1024}});
  add({{"lds_slots", 4096}});
  add({{"chunk_tiles", 1}});
  add({{"chunk_tiles", 4}});
  add({{"chunk_tiles", 16}});
  add({{"grid", static_cast<double>(cu)}});
  add({{"grid", static_cast<double>(2 * cu)}});
  // spilled rows of batched plans: device atomics instead of records, or
  // records over fewer or more partitions than the default
  add({{"fanout", -1}});
  add({{"fanout", 16}});
  add({{"fanout", 256}});
  return c;
}

// --------------------------------------------------------- device scratch

struct DeviceBuf {
  void* p = nullptr;
  ~DeviceBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) {
    if (p) (void)hipFree(p);
    p = nullptr;
    return hipMalloc(&p, bytes < 256 ? 256 : bytes);
  }
};

int elem_bytes(int32_t type) { return type == REL_I8 ? 1 : (type == REL_I32 ? 4 : 8); }

int32_t key_type(const rel_pipeline_desc& d, int k) {
  const rel_key_ref& kr = d.keys[k];
  return kr.src == REL_KEY_FACT ? d.fact[kr.col].type : d.dims[kr.col].payload.type;
}

// The groups of the last run on the host, rows sorted by key tuple, as one
// byte string per row (keys widened to int64, then the aggregate words).
std::vector<std::string> host_groups(const rel_pipeline_desc& d, const rel_outputs& o,
                                     int64_t groups, hipStream_t s, hipError_t& e) {
  std::vector<std::string> rows;
  e = hipSuccess;
  if (groups <= 0) return rows;
  std::vector<std::vector<int64_t>> cols;
  for (int k = 0; k < d.n_keys; ++k) {
    const int w = elem_bytes(key_type(d, k));
    std::vector<unsigned char> raw(static_cast<size_t>(groups) * w);
    e = hipMemcpyAsync(raw.data(), o.keys[k], raw.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return rows;
    std::vector<int64_t> v(static_cast<size_t>(groups));
    for (int64_t g = 0; g < groups; ++g) {
      if (w == 1) v[g] = reinterpret_cast<const int8_t*>(raw.data())[g];
      else if (w == 4) v[g] = reinterpret_cast<const int32_t*>(raw.data())[g];
      else v[g] = reinterpret_cast<const int64_t*>(raw.data())[g];
    }
    cols.push_back(std::move(v));
  }
  for (int a = 0; a < d.n_aggs; ++a) {
    std::vector<int64_t> v(static_cast<size_t>(groups));
    e = hipMemcpyAsync(v.data(), o.aggs[a], v.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return rows;
    cols.push_back(std::move(v));
  }
  std::vector<int64_t> order(static_cast<size_t>(groups));
  for (int64_t g = 0; g < groups; ++g) order[g] = g;
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    for (int k = 0; k < d.n_keys; ++k)
      if (cols[k][x] != cols[k][y]) return cols[k][x] < cols[k][y];
    return x < y;
  });
  for (int64_t g : order) {
    std::string r;
    for (const auto& c : cols) r.append(reinterpret_cast<const char*>(&c[g]), 8);
    rows.push_back(std::move(r));
  }
  return rows;
}

void rel_clear_error() { clear_last_error(); }

rel_status rel_fail(rel_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return static_cast<rel_status>(set_last_error(st, buf));
}

}  // namespace
}  // namespace rel

using namespace rel;

extern "C" {

rel_status rel_autotune(const rel_pipeline_desc* samples, int n, const char* cache_path) {
  rel_clear_error();
  if (!samples || n < 1) return rel_fail(REL_EINVAL, "autotune: no sample plans");
  if (!cache_path || !*cache_path) return rel_fail(REL_EINVAL, "autotune: no cache path");
  for (int i = 0; i < n; ++i) {
    if (rel_pipeline_batch_ws(&samples[i], 1) == 0)
      return rel_fail(REL_EINVAL, "autotune: sample %d is not a valid plan", i);
  }
  Json root;
  if (!read_cache(cache_path, root))
    return rel_fail(REL_EINVAL, "autotune: %s is not a tuning cache", cache_path);
  const std::string arch = arch_name();
  int cu = device_info().cu_count;
  const std::vector<rel_tuning> cands = candidates(cu);
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
    return rel_fail(REL_EDEVICE, "autotune: stream");
  std::unique_ptr<void, void (*)(void*)> stream_guard(
      s, [](void* p) { (void)hipStreamDestroy(static_cast<hipStream_t>(p)); });
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) return rel_fail(REL_EDEVICE, "autotune: events");
  auto destroy_events = [&]() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  };
  constexpr int kReps = 3;
  for (int i = 0; i < n; ++i) {
    rel_pipeline_desc d = samples[i];
    size_t ws_bytes = 0;
    for (const rel_tuning& t : cands) {
      d.tuning = &t;
      ws_bytes = std::max(ws_bytes, rel_pipeline_batch_ws(&d, 1));
    }
    const int64_t cap = d.max_groups > 0 ? d.max_groups : 1;
    DeviceBuf ws, outs[REL_MAX_KEYS + REL_MAX_AGGS], count;
    hipError_t e = ws.alloc(ws_bytes);
    for (int k = 0; e == hipSuccess && k < d.n_keys; ++k) e = outs[k].alloc(cap * 8);
    for (int a = 0; e == hipSuccess && a < d.n_aggs; ++a) e = outs[REL_MAX_KEYS + a].alloc(cap * 8);
    if (e == hipSuccess) e = count.alloc(8);
    if (e != hipSuccess) {
      destroy_events();
      return rel_fail(REL_EDEVICE, "autotune: device memory: %s", hipGetErrorString(e));
    }
    rel_outputs o;
    std::memset(&o, 0, sizeof o);
    for (int k = 0; k < d.n_keys; ++k) o.keys[k] = outs[k].p;
    for (int a = 0; a < d.n_aggs; ++a) o.aggs[a] = outs[REL_MAX_KEYS + a].p;
    o.cap = cap;
    o.d_groups = static_cast<int64_t*>(count.p);
    std::vector<std::string> ref;
    Json times;
    times.kind = Json::kObj;
    double best_ms = -1;
    int best = 0;
    for (size_t c = 0; c < cands.size(); ++c) {
      d.tuning = &cands[c];
      // one warm run whose groups every candidate must reproduce
      rel_status st = rel_pipeline_batch(&d, 1, &o, ws.p, ws_bytes, s);
      int64_t groups = 0;
      if (st == REL_OK) {
        e = hipMemcpyAsync(&groups, o.d_groups, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = REL_EDEVICE;
      }
      if (st != REL_OK) {
        destroy_events();
        return rel_fail(st, "autotune: sample %d, candidate %zu failed", i, c);
      }
      if (groups < 0 || groups > cap) {
        destroy_events();
        return rel_fail(REL_ECAPACITY, "autotune: sample %d has more groups than max_groups", i);
      }
      std::vector<std::string> got = host_groups(d, o, groups, s, e);
      if (e != hipSuccess) {
        destroy_events();
        return rel_fail(REL_EDEVICE, "autotune: result copy: %s", hipGetErrorString(e));
      }
      if (c == 0) {
        ref = std::move(got);
      } else if (got != ref) {
        destroy_events();
        return rel_fail(REL_EDEVICE,
                        "autotune: sample %d: candidate %s changed the result (a race)", i,
                        compact(record_of(cands[c])).c_str());
      }
      e = hipEventRecord(ev[0], s);
      for (int r = 0; e == hipSuccess && r < kReps; ++r)
        if (rel_pipeline_batch(&d, 1, &o, ws.p, ws_bytes, s) != REL_OK) e = hipErrorUnknown;
      if (e == hipSuccess) e = hipEventRecord(ev[1], s);
      if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
      if (e != hipSuccess) {
        destroy_events();
        return rel_fail(REL_EDEVICE, "autotune: timing: %s", hipGetErrorString(e));
      }
      const double per = ms / kReps;
      times.obj[compact(record_of(cands[c]))] = number(std::round(per * 1e4) / 1e4);
      if (best_ms < 0 || per < best_ms) {
        best_ms = per;
        best = static_cast<int>(c);
      }
    }
    Json rec;
    rec.kind = Json::kObj;
    rec.obj["tuning"] = record_of(cands[best]);
    rec.obj["ms"] = number(std::round(best_ms * 1e4) / 1e4);
    rec.obj["candidates"] = times;
    root.obj[cache_key(arch, samples[i])] = rec;
  }
  destroy_events();
  if (!write_cache(cache_path, root))
    return rel_fail(REL_EINVAL, "autotune: cannot write %s", cache_path);
  return REL_OK;
}

rel_status rel_autotune_lookup(const char* cache_path, const rel_pipeline_desc* d,
                               rel_tuning* out, int* found) {
  rel_clear_error();
  if (!cache_path || !d || !out || !found) return rel_fail(REL_EINVAL, "autotune lookup: NULL argument");
  if (!d->fact || d->n_fact < 1) return rel_fail(REL_EINVAL, "autotune lookup: no fact columns");
  if (d->n_dims > 0 && !d->dims) return rel_fail(REL_EINVAL, "autotune lookup: NULL dims");
  *found = 0;
  std::memset(out, 0, sizeof *out);
  Json root;
  if (!read_cache(cache_path, root))
    return rel_fail(REL_EINVAL, "autotune lookup: %s is not a tuning cache", cache_path);
  auto it = root.obj.find(cache_key(arch_name(), *d));
  if (it == root.obj.end()) return REL_OK;
  auto t = it->second.obj.find("tuning");
  if (t == it->second.obj.end() || t->second.kind != Json::kObj)
    return rel_fail(REL_EINVAL, "autotune lookup: record without a tuning");
  for (const auto& kv : t->second.obj) {
    bool known = false;
    for (const Field& f : kFields) known |= kv.first == f.name;
    if (!known || kv.second.kind != Json::kNum)
      return rel_fail(REL_EINVAL, "autotune lookup: unknown tuning field %s", kv.first.c_str());
    set_field(*out, kv.first, kv.second.num);
  }
  *found = 1;
  return REL_OK;
}

}  // extern "C"
