// A small JSON reader for the tuning file: objects, arrays, strings (with the
// standard escapes), numbers, true / false / null, nested at most 64 deep.
// Anything outside JSON's grammar (a bad escape, a hex / inf / nan number, a
// number that overflows double, trailing text) fails the parse.
#pragma once

#include <cmath>
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
  static int hexval(char c) {
    if (c >= '0' && c <= '9') return c - '0';
    if (c >= 'a' && c <= 'f') return c - 'a' + 10;
    if (c >= 'A' && c <= 'F') return c - 'A' + 10;
    return -1;
  }
  bool digit() const { return i_ < s_.size() && s_[i_] >= '0' && s_[i_] <= '9'; }
  // A number in JSON's grammar, -?(0|[1-9][0-9]*)(.[0-9]+)?([eE][+-]?[0-9]+)?;
  // no hex, inf or nan spellings, and a finite value.
  void number(Value* v) {
    const size_t start = i_;
    if (i_ < s_.size() && s_[i_] == '-') ++i_;
    if (!digit()) {
      ok_ = false;
      return;
    }
    if (s_[i_] == '0') {
      ++i_;
    } else {
      while (digit()) ++i_;
    }
    if (i_ < s_.size() && s_[i_] == '.') {
      ++i_;
      if (!digit()) {
        ok_ = false;
        return;
      }
      while (digit()) ++i_;
    }
    if (i_ < s_.size() && (s_[i_] == 'e' || s_[i_] == 'E')) {
      ++i_;
      if (i_ < s_.size() && (s_[i_] == '+' || s_[i_] == '-')) ++i_;
      if (!digit()) {
        ok_ = false;
        return;
      }
      while (digit()) ++i_;
    }
    const std::string text = s_.substr(start, i_ - start);
    const double d = std::strtod(text.c_str(), nullptr);
    if (!std::isfinite(d)) {
      ok_ = false;
      return;
    }
    v->kind = Value::Number;
    v->num = d;
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
          case 'u': {  // exactly four hex digits; ASCII kept, other code points become '?'
            long cp = 0;
            for (int d = 0; d < 4; ++d) {
              const int h = i_ + d < s_.size() ? hexval(s_[i_ + d]) : -1;
              if (h < 0) {
                ok_ = false;
                return;
              }
              cp = cp * 16 + h;
            }
            i_ += 4;
            c = cp < 128 ? (char)cp : '?';
            break;
          }
          case '"': case '\\': case '/': c = e; break;
          default:  // not a JSON escape
            ok_ = false;
            return;
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
      number(v);
    }
  }
};

}  // namespace json
}  // namespace stockfft
