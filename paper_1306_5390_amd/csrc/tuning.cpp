// tuning.cpp -- the tuning cache file: which kernel shape the fused path and
// the batch path use for each beta and image size class.  A small JSON
// document, written by phgrms_save_tuning / phgrms_autotune and by the
// Python autotuner (which adds its measured rates), read by
// phgrms_load_tuning and phgrms_batch_plan.
//
//   {"format": "phgrms-tuning-1",
//    "shapes": [[T, rows, waves], ...],        // compiled shapes, by index
//    "choice": {"<beta>": {"<class>": {"shape": s, ...}, ...}, ...},
//    "batch_choice": {"<beta>": {"shape": s, "classes": {"<class>": s}}, ...}}
//
// Every field is optional; entries that are absent keep the current value.
// A batch entry's "shape" applies to every size class, "classes" overrides
// single classes.  Other keys (rates, notes) are ignored when reading and
// kept when the file is rewritten.
#include <algorithm>
#include <cctype>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "phgrms.h"
#include "host_common.hpp"

namespace phg {

namespace {

struct Json {
  enum Kind { Null, Bool, Num, Str, Arr, Obj } kind = Null;
  bool b = false;
  double num = 0.0;
  std::string str;
  std::vector<Json> arr;
  std::vector<std::pair<std::string, Json>> obj;
  const Json* get(const std::string& key) const {
    if (kind != Obj) return nullptr;
    for (const auto& kv : obj)
      if (kv.first == key) return &kv.second;
    return nullptr;
  }
};

// Recursive-descent reader of one JSON value (RFC 8259 grammar).
class Reader {
 public:
  explicit Reader(const std::string& s) : s_(s) {}
  bool parse(Json& out) {
    if (!value(out, 0)) return false;
    ws();
    if (i_ != s_.size()) return err("trailing characters");
    return true;
  }
  size_t pos() const { return i_; }
  const char* what() const { return what_; }

 private:
  const std::string& s_;
  size_t i_ = 0;
  const char* what_ = "";

  bool err(const char* w) {
    what_ = w;
    return false;
  }
  void ws() {
    while (i_ < s_.size() && (s_[i_] == ' ' || s_[i_] == '\t' || s_[i_] == '\n' || s_[i_] == '\r'))
      ++i_;
  }
  bool lit(const char* w) {
    const size_t n = std::strlen(w);
    if (s_.compare(i_, n, w) != 0) return err("bad literal");
    i_ += n;
    return true;
  }
  bool string(std::string& out) {
    if (i_ >= s_.size() || s_[i_] != '"') return err("expected a string");
    ++i_;
    out.clear();
    while (i_ < s_.size() && s_[i_] != '"') {
      char c = s_[i_++];
      if (static_cast<unsigned char>(c) < 0x20) return err("control character in a string");
      if (c == '\\') {
        if (i_ >= s_.size()) return err("unterminated escape");
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
            uint32_t cp = 0;
            if (!hex4(cp)) return false;
            if (cp >= 0xD800 && cp < 0xDC00 && i_ + 6 <= s_.size() && s_[i_] == '\\' &&
                s_[i_ + 1] == 'u') {
              i_ += 2;
              uint32_t lo = 0;
              if (!hex4(lo)) return false;
              if (lo < 0xDC00 || lo >= 0xE000) return err("bad surrogate pair");
              cp = 0x10000 + ((cp - 0xD800) << 10) + (lo - 0xDC00);
            }
            utf8(cp, out);
            continue;
          }
          default: return err("bad escape");
        }
      }
      out += c;
    }
    if (i_ >= s_.size()) return err("unterminated string");
    ++i_;
    return true;
  }
  bool hex4(uint32_t& v) {
    if (i_ + 4 > s_.size()) return err("short \\u escape");
    v = 0;
    for (int k = 0; k < 4; ++k) {
      const char h = s_[i_++];
      v <<= 4;
      if (h >= '0' && h <= '9') v |= uint32_t(h - '0');
      else if (h >= 'a' && h <= 'f') v |= uint32_t(h - 'a' + 10);
      else if (h >= 'A' && h <= 'F') v |= uint32_t(h - 'A' + 10);
      else return err("bad \\u escape");
    }
    return true;
  }
  static void utf8(uint32_t cp, std::string& out) {
    if (cp < 0x80) {
      out += char(cp);
    } else if (cp < 0x800) {
      out += char(0xC0 | (cp >> 6));
      out += char(0x80 | (cp & 0x3F));
    } else if (cp < 0x10000) {
      out += char(0xE0 | (cp >> 12));
      out += char(0x80 | ((cp >> 6) & 0x3F));
      out += char(0x80 | (cp & 0x3F));
    } else {
      out += char(0xF0 | (cp >> 18));
      out += char(0x80 | ((cp >> 12) & 0x3F));
      out += char(0x80 | ((cp >> 6) & 0x3F));
      out += char(0x80 | (cp & 0x3F));
    }
  }
  bool number(double& v) {
    const size_t b = i_;
    if (i_ < s_.size() && s_[i_] == '-') ++i_;
    while (i_ < s_.size() && (std::isdigit(static_cast<unsigned char>(s_[i_])) || s_[i_] == '.' ||
                              s_[i_] == 'e' || s_[i_] == 'E' || s_[i_] == '+' || s_[i_] == '-'))
      ++i_;
    if (i_ == b) return err("expected a value");
    const std::string t = s_.substr(b, i_ - b);
    char* end = nullptr;
    errno = 0;
    v = std::strtod(t.c_str(), &end);
    if (end == nullptr || *end != '\0' || errno == ERANGE) return err("bad number");
    return true;
  }
  bool value(Json& out, int depth) {
    if (depth > 64) return err("nesting too deep");
    ws();
    if (i_ >= s_.size()) return err("unexpected end");
    const char c = s_[i_];
    if (c == '{') {
      out.kind = Json::Obj;
      ++i_;
      ws();
      if (i_ < s_.size() && s_[i_] == '}') {
        ++i_;
        return true;
      }
      for (;;) {
        ws();
        std::string key;
        if (!string(key)) return false;
        ws();
        if (i_ >= s_.size() || s_[i_] != ':') return err("expected ':'");
        ++i_;
        Json v;
        if (!value(v, depth + 1)) return false;
        out.obj.emplace_back(std::move(key), std::move(v));
        ws();
        if (i_ < s_.size() && s_[i_] == ',') {
          ++i_;
          continue;
        }
        if (i_ < s_.size() && s_[i_] == '}') {
          ++i_;
          return true;
        }
        return err("expected ',' or '}'");
      }
    }
    if (c == '[') {
      out.kind = Json::Arr;
      ++i_;
      ws();
      if (i_ < s_.size() && s_[i_] == ']') {
        ++i_;
        return true;
      }
      for (;;) {
        Json v;
        if (!value(v, depth + 1)) return false;
        out.arr.push_back(std::move(v));
        ws();
        if (i_ < s_.size() && s_[i_] == ',') {
          ++i_;
          continue;
        }
        if (i_ < s_.size() && s_[i_] == ']') {
          ++i_;
          return true;
        }
        return err("expected ',' or ']'");
      }
    }
    if (c == '"') {
      out.kind = Json::Str;
      return string(out.str);
    }
    if (c == 't') {
      out.kind = Json::Bool;
      out.b = true;
      return lit("true");
    }
    if (c == 'f') {
      out.kind = Json::Bool;
      return lit("false");
    }
    if (c == 'n') return lit("null");
    out.kind = Json::Num;
    return number(out.num);
  }
};

void dump_string(const std::string& v, std::string& o) {
  o += '"';
  for (char c : v) {
    if (c == '"' || c == '\\') {
      o += '\\';
      o += c;
    } else if (static_cast<unsigned char>(c) < 0x20) {
      char b[8];
      std::snprintf(b, sizeof(b), "\\u%04x", unsigned(static_cast<unsigned char>(c)));
      o += b;
    } else {
      o += c;
    }
  }
  o += '"';
}

// JSON text of v; objects one key per line at the outer two levels.
void dump(const Json& v, std::string& o, int depth) {
  char b[64];
  switch (v.kind) {
    case Json::Null: o += "null"; return;
    case Json::Bool: o += v.b ? "true" : "false"; return;
    case Json::Num:
      if (std::floor(v.num) == v.num && std::fabs(v.num) < 9.007199254740992e15)
        std::snprintf(b, sizeof(b), "%.0f", v.num);
      else
        std::snprintf(b, sizeof(b), "%.17g", v.num);
      o += b;
      return;
    case Json::Str: dump_string(v.str, o); return;
    case Json::Arr:
      o += '[';
      for (size_t i = 0; i < v.arr.size(); ++i) {
        if (i) o += ", ";
        dump(v.arr[i], o, depth + 1);
      }
      o += ']';
      return;
    case Json::Obj: {
      const bool lines = depth < 2;
      o += '{';
      for (size_t i = 0; i < v.obj.size(); ++i) {
        o += i ? "," : "";
        if (lines) {
          o += '\n';
          o.append(size_t(depth + 1), ' ');
        } else if (i) {
          o += ' ';
        }
        dump_string(v.obj[i].first, o);
        o += ": ";
        dump(v.obj[i].second, o, depth + 1);
      }
      if (lines && !v.obj.empty()) {
        o += '\n';
        o.append(size_t(depth), ' ');
      }
      o += '}';
      return;
    }
  }
}

Json number(double x) {
  Json j;
  j.kind = Json::Num;
  j.num = x;
  return j;
}

// The member `key` of object o, created (as an empty object) if missing or
// not an object.  The reference is valid until o gains another member.
Json& member(Json& o, const std::string& key) {
  for (auto& kv : o.obj)
    if (kv.first == key) {
      if (kv.second.kind != Json::Obj) {
        kv.second = Json();
        kv.second.kind = Json::Obj;
      }
      return kv.second;
    }
  Json e;
  e.kind = Json::Obj;
  o.obj.emplace_back(key, std::move(e));
  return o.obj.back().second;
}

void set_member(Json& o, const std::string& key, Json v) {
  for (auto& kv : o.obj)
    if (kv.first == key) {
      kv.second = std::move(v);
      return;
    }
  o.obj.emplace_back(key, std::move(v));
}

bool read_text(const char* path, std::string& text, bool& missing) {
  missing = false;
  std::unique_ptr<FILE, int (*)(FILE*)> f(std::fopen(path, "rb"), &std::fclose);
  if (!f) {
    missing = errno == ENOENT;
    fail(missing ? PHGRMS_ENOTFOUND : PHGRMS_EINVAL, "cannot open tuning cache %s: %s", path,
         std::strerror(errno));
    return false;
  }
  char buf[65536];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f.get())) > 0) {
    text.append(buf, got);
    if (text.size() > (size_t(16) << 20)) {
      fail(PHGRMS_EINVAL, "tuning cache %s over 16 MiB", path);
      return false;
    }
  }
  if (std::ferror(f.get())) {
    fail(PHGRMS_EINVAL, "cannot read tuning cache %s", path);
    return false;
  }
  return true;
}

// A non-negative integer key ("1", "2", ...) or -1.
int int_key(const std::string& k) {
  if (k.empty() || k.size() > 6) return -1;
  int v = 0;
  for (char c : k) {
    if (c < '0' || c > '9') return -1;
    v = v * 10 + (c - '0');
  }
  return v;
}

// The integer value of a "shape" number, or -1.
int shape_value(const Json* v) {
  if (v == nullptr || v->kind != Json::Num) return -1;
  const double d = v->num;
  if (!(d >= 0.0 && d < double(kNumShapes)) || std::floor(d) != d) return -1;
  return int(d);
}

}  // namespace

namespace {

int parse_tuning(const char* path, const std::string& text, TuneTables& t, Json& root) {
  Reader rd(text);
  if (!rd.parse(root)) return fail(PHGRMS_EINVAL, "tuning cache %s: %s at byte %zu", path, rd.what(), rd.pos());
  if (root.kind != Json::Obj) return fail(PHGRMS_EINVAL, "tuning cache %s: not a JSON object", path);
  TuneTables n = t;
  // The shapes the file's indices refer to must be the compiled ones.
  if (const Json* sh = root.get("shapes")) {
    if (sh->kind != Json::Arr) return fail(PHGRMS_EINVAL, "tuning cache %s: \"shapes\" is not a list", path);
    for (size_t i = 0; i < sh->arr.size(); ++i) {
      const Json& e = sh->arr[i];
      if (e.kind != Json::Arr || e.arr.size() < 3)
        return fail(PHGRMS_EINVAL, "tuning cache %s: shape %zu is not [T, rows, waves]", path, i);
      if (int(i) >= kNumShapes) break;   // shapes the library does not have are never chosen below
      const int want[3] = {kShapes[i].T, kShapes[i].rows, kShapes[i].waves};
      for (int j = 0; j < 3; ++j)
        if (e.arr[j].kind != Json::Num || e.arr[j].num != double(want[j]))
          return fail(PHGRMS_EINVAL, "tuning cache %s: shape %zu differs from the compiled one", path, i);
    }
  }
  if (const Json* ch = root.get("choice")) {
    if (ch->kind != Json::Obj) return fail(PHGRMS_EINVAL, "tuning cache %s: \"choice\" is not an object", path);
    for (const auto& bk : ch->obj) {
      const int beta = int_key(bk.first);
      if (beta < 1 || beta > PHGRMS_BETA_MAX || bk.second.kind != Json::Obj)
        return fail(PHGRMS_EINVAL, "tuning cache %s: bad choice entry \"%s\"", path, bk.first.c_str());
      for (const auto& ck : bk.second.obj) {
        const int cls = int_key(ck.first);
        const int s = shape_value(ck.second.get("shape"));
        if (cls < 0 || cls >= kSizeClasses || s < 0)
          return fail(PHGRMS_EINVAL, "tuning cache %s: bad choice for beta %d class \"%s\"", path, beta,
                      ck.first.c_str());
        n.fused[beta][cls] = s;
      }
    }
  }
  if (const Json* bc = root.get("batch_choice")) {
    if (bc->kind != Json::Obj)
      return fail(PHGRMS_EINVAL, "tuning cache %s: \"batch_choice\" is not an object", path);
    for (const auto& bk : bc->obj) {
      const int beta = int_key(bk.first);
      if (beta < 0) continue;   // notes and other keys
      if (beta < 1 || beta > PHGRMS_BETA_MAX || bk.second.kind != Json::Obj)
        return fail(PHGRMS_EINVAL, "tuning cache %s: bad batch entry \"%s\"", path, bk.first.c_str());
      if (const Json* v = bk.second.get("shape")) {
        const int s = shape_value(v);
        if (s < 0) return fail(PHGRMS_EINVAL, "tuning cache %s: bad batch shape for beta %d", path, beta);
        for (int c = 0; c < kSizeClasses; ++c) n.batch[beta][c] = s;
      }
      if (const Json* cl = bk.second.get("classes")) {
        if (cl->kind != Json::Obj)
          return fail(PHGRMS_EINVAL, "tuning cache %s: bad batch classes for beta %d", path, beta);
        for (const auto& ck : cl->obj) {
          const int cls = int_key(ck.first);
          const int s = shape_value(&ck.second);
          if (cls < 0 || cls >= kSizeClasses || s < 0)
            return fail(PHGRMS_EINVAL, "tuning cache %s: bad batch class \"%s\" for beta %d", path,
                        ck.first.c_str(), beta);
          n.batch[beta][cls] = s;
        }
      }
    }
  }
  t = n;
  return PHGRMS_OK;
}

}  // namespace

int read_tuning_file(const char* path, TuneTables& t) {
  if (path == nullptr || path[0] == '\0') return fail(PHGRMS_EINVAL, "null tuning cache path");
  std::string text;
  bool missing = false;
  if (!read_text(path, text, missing)) return missing ? PHGRMS_ENOTFOUND : PHGRMS_EINVAL;
  Json root;
  return parse_tuning(path, text, t, root);
}

int write_tuning_file(const char* path, const TuneTables& t) {
  if (path == nullptr || path[0] == '\0') return fail(PHGRMS_EINVAL, "null tuning cache path");
  // Start from the file's own document when there is a valid one, so that
  // keys this library does not use (measured rates, notes) survive.
  Json root;
  root.kind = Json::Obj;
  {
    std::string text;
    bool missing = false;
    if (read_text(path, text, missing)) {
      TuneTables scratch = t;
      Json doc;
      if (parse_tuning(path, text, scratch, doc) != PHGRMS_OK)
        return fail(PHGRMS_EINVAL, "tuning cache %s exists and is not a valid cache; not overwritten",
                    path);
      root = std::move(doc);
    } else if (!missing) {
      return PHGRMS_EINVAL;
    }
  }
  Json fmt;
  fmt.kind = Json::Str;
  fmt.str = "phgrms-tuning-1";
  set_member(root, "format", fmt);
  Json shapes;
  shapes.kind = Json::Arr;
  for (int i = 0; i < kNumShapes; ++i) {
    Json e;
    e.kind = Json::Arr;
    e.arr = {number(kShapes[i].T), number(kShapes[i].rows), number(kShapes[i].waves)};
    shapes.arr.push_back(std::move(e));
  }
  set_member(root, "shapes", std::move(shapes));
  // (both members first: adding one may move the other)
  member(root, "choice");
  member(root, "batch_choice");
  Json& choice = member(root, "choice");
  Json& batch = member(root, "batch_choice");
  for (int b = 1; b <= PHGRMS_BETA_MAX; ++b) {
    Json& cb = member(choice, std::to_string(b));
    for (int c = 0; c < kSizeClasses; ++c)
      set_member(member(cb, std::to_string(c)), "shape", number(t.fused[b][c]));
    Json& bb = member(batch, std::to_string(b));
    // per class; a single "shape" would override them on reading
    bb.obj.erase(std::remove_if(bb.obj.begin(), bb.obj.end(),
                                [](const std::pair<std::string, Json>& kv) { return kv.first == "shape"; }),
                 bb.obj.end());
    Json& cl = member(bb, "classes");
    for (int c = 0; c < kSizeClasses; ++c) set_member(cl, std::to_string(c), number(t.batch[b][c]));
  }
  std::string o;
  dump(root, o, 0);
  o += '\n';
  // write a sibling file, then rename over the target (readers never see a
  // partial file)
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::unique_ptr<FILE, int (*)(FILE*)> f(std::fopen(tmp.c_str(), "wb"), &std::fclose);
    if (!f) return fail(PHGRMS_EINVAL, "cannot write tuning cache %s: %s", tmp.c_str(), std::strerror(errno));
    if (std::fwrite(o.data(), 1, o.size(), f.get()) != o.size() || std::fflush(f.get()) != 0)
      return fail(PHGRMS_EINVAL, "cannot write tuning cache %s", tmp.c_str());
  }
  if (std::rename(tmp.c_str(), path) != 0)
    return fail(PHGRMS_EINVAL, "cannot rename %s to %s: %s", tmp.c_str(), path, std::strerror(errno));
  return PHGRMS_OK;
}

}  // namespace phg
