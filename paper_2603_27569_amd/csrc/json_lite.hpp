// A small JSON reader for the tuning file: objects, arrays, strings (with the
// standard escapes), numbers, true / false / null.  Parse errors leave the
// value of kind Null and set ok = false.
#pragma once

#include <cstdlib>
#include <map>
#include <memory>
#include <string>
#include <vector>

namespace stockfft {
namespace json {

struct Value {
  enum Kind { Null, Bool, Number, String, Array, Object } kind = Null;
  bool b = false;
  double num = 0.0;
  std::string str;
  std::vector<Value> arr;
  std::map<std::string, Value> obj;

  const Value* get(const std::string& key) const {
    if (kind != Object) return nullptr;
    auto it = obj.find(key);
    return it == obj.end() ? nullptr : &it->second;
  }
};

class Parser {
 public:
  explicit Parser(const std::string& text) : s_(text) {}

  bool parse(Value* out) {
    ok_ = true;
    value(out, 0);
    ws();
    if (i_ != s_.size()) ok_ = false;
    return ok_;
  }

 private:
  const std::string& s_;
  size_t i_ = 0;
  bool ok_ = true;

  void ws() {
    while (i_ < s_.size() && (s_[i_] == ' ' || s_[i_] == '\n' || s_[i_] == '\r' || s_[i_] == '\t'))
      ++i_;
  }
  bool eat(char c) {
    ws();
    if (i_ < s_.size() && s_[i_] == c) {
      ++i_;
      return true;
    }
    return false;
  }
  bool lit(const char* w) {
    size_t n = std::char_traits<char>::length(w);
    if (s_.compare(i_, n, w) == 0) {
      i_ += n;
      return true;
    }
    return false;
  }
  void string(std::string* out) {
    // caller consumed the opening quote
    while (i_ < s_.size() && s_[i_] != '"') {
      char c = s_[i_++];
      if (c == '\\') {
        if (i_ >= s_.size()) break;
        char e = s_[i_++];
        switch (e) {
          case 'n': c = '\n'; break;
          case 't': c = '\t'; break;
          case 'r': c = '\r'; break;
          case 'b': c = '\b'; break;
          case 'f': c = '\f'; break;
          case 'u':  // keep ASCII only; other code points become '?'
            if (i_ + 4 <= s_.size()) {
              long cp = std::strtol(s_.substr(i_, 4).c_str(), nullptr, 16);
              c = cp < 128 ? (char)cp : '?';
              i_ += 4;
            } else {
              ok_ = false;
            }
            break;
          default: c = e;
        }
      }
      out->push_back(c);
    }
    if (i_ >= s_.size()) {
      ok_ = false;
      return;
    }
    ++i_;  // closing quote
  }
  void value(Value* v, int depth) {
    if (depth > 64) {
      ok_ = false;
      return;
    }
    ws();
    if (i_ >= s_.size()) {
      ok_ = false;
      return;
    }
    const char c = s_[i_];
    if (c == '{') {
      ++i_;
      v->kind = Value::Object;
      if (eat('}')) return;
      do {
        if (!eat('"')) {
          ok_ = false;
          return;
        }
        std::string key;
        string(&key);
        if (!eat(':')) {
          ok_ = false;
          return;
        }
        value(&v->obj[key], depth + 1);
        if (!ok_) return;
      } while (eat(','));
      if (!eat('}')) ok_ = false;
    } else if (c == '[') {
      ++i_;
      v->kind = Value::Array;
      if (eat(']')) return;
      do {
        v->arr.emplace_back();
        value(&v->arr.back(), depth + 1);
        if (!ok_) return;
      } while (eat(','));
      if (!eat(']')) ok_ = false;
    } else if (c == '"') {
      ++i_;
      v->kind = Value::String;
      string(&v->str);
    } else if (lit("true")) {
      v->kind = Value::Bool;
      v->b = true;
    } else if (lit("false")) {
      v->kind = Value::Bool;
    } else if (lit("null")) {
      v->kind = Value::Null;
    } else {
      const char* start = s_.c_str() + i_;
      char* end = nullptr;
      v->num = std::strtod(start, &end);
      if (end == start) {
        ok_ = false;
        return;
      }
      v->kind = Value::Number;
      i_ += (size_t)(end - start);
    }
  }
};

}  // namespace json
}  // namespace stockfft
