// Front end: error reporting, dtype tables, the argument-signature parser,
// a C tokenizer and the expression classifier.
//
// The user's C argument list and statement / map expression are taken as
// text (section "Efficient Evaluation of Element-wise Expressions": "a
// C-style argument list and a statement (or semicolon-separated list of
// statements) to be executed for each value of i"; section "Map-Reduce":
// result dtype first, then arguments, map, reduce and neutral expressions).
// The classifier decides which arrays a kernel must load and store and
// whether the 16-byte vector kernel applies (every array access is exactly
// name[i]).
#include <cctype>
#include <cstring>
#include <map>
#include <set>

#include "common.h"

namespace hipmr {

// ---------------------------------------------------------------- errors
namespace {
thread_local std::string g_last_error;
}

hipmr_status fail(hipmr_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}
void clear_error() { g_last_error.clear(); }
const char* last_error() { return g_last_error.c_str(); }

// ---------------------------------------------------------------- dtypes
int dtype_size(DType t) {
    switch (t) {
        case DT_F32: case DT_I32: case DT_U32: return 4;
        case DT_F64: case DT_I64: case DT_C64: return 8;
        case DT_I16: case DT_U16: case DT_BF16: case DT_F16: return 2;
        case DT_I8: case DT_U8: case DT_FP8: return 1;
        default: return 0;
    }
}

const char* dtype_device_name(DType t) {
    switch (t) {
        case DT_F32: return "float";
        case DT_F64: return "double";
        case DT_I8: return "signed char";
        case DT_U8: return "unsigned char";
        case DT_I16: return "short";
        case DT_U16: return "unsigned short";
        case DT_I32: return "int";
        case DT_U32: return "unsigned int";
        case DT_I64: return "long long";
        case DT_BF16: return "hipmr_bf16";
        case DT_F16: return "hipmr_f16";
        case DT_FP8: return "hipmr_fp8";
        case DT_C64: return "hipmr_c64";
        default: return "void";
    }
}

bool dtype_is_float(DType t) {
    return t == DT_F32 || t == DT_F64 || t == DT_BF16 || t == DT_F16 || t == DT_FP8;
}
bool dtype_is_lowp(DType t) { return t == DT_BF16 || t == DT_F16 || t == DT_FP8; }

namespace {

const std::map<std::string, DType>& type_words() {
    static const std::map<std::string, DType> m = {
        {"float", DT_F32}, {"double", DT_F64},
        {"int8_t", DT_I8}, {"char", DT_I8}, {"signed char", DT_I8},
        {"uint8_t", DT_U8}, {"unsigned char", DT_U8},
        {"int16_t", DT_I16}, {"short", DT_I16}, {"short int", DT_I16},
        {"uint16_t", DT_U16}, {"unsigned short", DT_U16},
        {"int32_t", DT_I32}, {"int", DT_I32}, {"signed", DT_I32}, {"signed int", DT_I32},
        {"uint32_t", DT_U32}, {"unsigned", DT_U32}, {"unsigned int", DT_U32},
        {"int64_t", DT_I64}, {"long", DT_I64}, {"long int", DT_I64}, {"long long", DT_I64},
        {"long long int", DT_I64},
        {"bfloat16", DT_BF16}, {"__hip_bfloat16", DT_BF16},
        {"half", DT_F16}, {"__half", DT_F16}, {"float16", DT_F16}, {"_Float16", DT_F16},
        {"fp8_e4m3", DT_FP8},
        {"complex64", DT_C64}, {"cfloat", DT_C64},
    };
    return m;
}

std::string trim(const std::string& s) {
    size_t a = 0, b = s.size();
    while (a < b && std::isspace((unsigned char)s[a])) ++a;
    while (b > a && std::isspace((unsigned char)s[b - 1])) --b;
    return s.substr(a, b - a);
}

bool is_ident_start(char c) { return std::isalpha((unsigned char)c) || c == '_'; }

// Generated kernels name everything they declare hipmr_* / HIPMR_*.
bool has_reserved_prefix(const std::string& name) {
    if (name.size() < 6) return false;
    std::string p = name.substr(0, 6);
    for (char& c : p) c = (char)std::tolower((unsigned char)c);
    return p == "hipmr_";
}
bool is_ident_char(char c) { return std::isalnum((unsigned char)c) || c == '_'; }

}  // namespace

// ---------------------------------------------------------------- signature
hipmr_status parse_signature(const std::string& text, Signature* out) {
    *out = Signature();
    std::string rest = text;
    size_t colon = text.find(':');
    if (colon != std::string::npos) {
        std::string head = trim(text.substr(0, colon));
        // collapse internal whitespace runs
        std::string norm;
        for (char c : head) {
            if (std::isspace((unsigned char)c)) {
                if (!norm.empty() && norm.back() != ' ') norm += ' ';
            } else {
                norm += c;
            }
        }
        auto it = type_words().find(norm);
        if (it == type_words().end())
            return fail(HIPMR_E_PARSE, "signature: unknown result type '" + head + "'");
        out->is_reduce = true;
        out->result = it->second;
        rest = text.substr(colon + 1);
    }
    if (trim(rest).empty()) return HIPMR_OK;
    size_t start = 0;
    std::set<std::string> seen;
    while (start <= rest.size()) {
        size_t comma = rest.find(',', start);
        std::string decl = trim(rest.substr(start, comma == std::string::npos ? std::string::npos
                                                                             : comma - start));
        start = comma == std::string::npos ? rest.size() + 1 : comma + 1;
        // split into words and '*'
        std::vector<std::string> words;
        for (size_t k = 0; k < decl.size();) {
            char c = decl[k];
            if (std::isspace((unsigned char)c)) { ++k; continue; }
            if (c == '*') { words.push_back("*"); ++k; continue; }
            if (is_ident_start(c)) {
                size_t j = k;
                while (j < decl.size() && is_ident_char(decl[j])) ++j;
                words.push_back(decl.substr(k, j - k));
                k = j;
                continue;
            }
            return fail(HIPMR_E_PARSE, "signature: unexpected '" + std::string(1, c) +
                                           "' in declaration '" + decl + "'");
        }
        ArgDecl a;
        std::vector<std::string> tw;
        for (size_t k = 0; k + 1 < words.size(); ++k) {
            const std::string& w = words[k];
            if (w == "const") { a.is_const = true; continue; }
            if (w == "__restrict__" || w == "restrict") continue;
            if (w == "*") {
                if (a.pointer) return fail(HIPMR_E_UNSUPPORTED, "signature: pointer to pointer in '" + decl + "'");
                a.pointer = true;
                continue;
            }
            if (a.pointer) return fail(HIPMR_E_PARSE, "signature: bad declaration '" + decl + "'");
            tw.push_back(w);
        }
        if (words.empty() || !is_ident_start(words.back()[0]) || tw.empty())
            return fail(HIPMR_E_PARSE, "signature: bad declaration '" + decl + "'");
        a.name = words.back();
        std::string type;
        for (auto& w : tw) type += (type.empty() ? "" : " ") + w;
        auto it = type_words().find(type);
        if (it == type_words().end())
            return fail(HIPMR_E_PARSE, "signature: unknown type '" + type + "' in '" + decl + "'");
        a.dtype = it->second;
        if (a.name == "i" || a.name == "n")
            return fail(HIPMR_E_PARSE, "signature: '" + a.name + "' is reserved (formal index / length)");
        if (has_reserved_prefix(a.name))
            return fail(HIPMR_E_PARSE, "signature: names starting with hipmr_ (any case) are reserved");
        if (!seen.insert(a.name).second)
            return fail(HIPMR_E_PARSE, "signature: duplicate argument '" + a.name + "'");
        out->args.push_back(a);
    }
    return HIPMR_OK;
}

// ---------------------------------------------------------------- lexer
hipmr_status lex(const std::string& src, std::vector<Token>* out) {
    static const char* punct[] = {"<<=", ">>=", "->", "++", "--", "<<", ">>", "<=", ">=",
                                  "==", "!=", "&&", "||", "+=", "-=", "*=", "/=", "%=",
                                  "&=", "|=", "^=", "::", "+", "-", "*", "/", "%", "<",
                                  ">", "=", "!", "~", "&", "|", "^", "?", ":", ",", ";",
                                  "(", ")", "[", "]", "{", "}", ".", nullptr};
    out->clear();
    size_t k = 0, n = src.size();
    while (k < n) {
        char c = src[k];
        if (std::isspace((unsigned char)c)) { ++k; continue; }
        if (src.compare(k, 2, "//") == 0) {
            size_t j = src.find('\n', k);
            k = j == std::string::npos ? n : j + 1;
            continue;
        }
        if (src.compare(k, 2, "/*") == 0) {
            size_t j = src.find("*/", k + 2);
            if (j == std::string::npos) return fail(HIPMR_E_PARSE, "expression: unterminated comment");
            k = j + 2;
            continue;
        }
        if (is_ident_start(c)) {
            size_t j = k + 1;
            while (j < n && is_ident_char(src[j])) ++j;
            out->push_back({Token::Ident, src.substr(k, j - k), k});
            k = j;
            continue;
        }
        if (std::isdigit((unsigned char)c) || (c == '.' && k + 1 < n && std::isdigit((unsigned char)src[k + 1]))) {
            size_t j = k;
            while (j < n) {
                char d = src[j];
                if (is_ident_char(d) || d == '.') { ++j; continue; }
                if ((d == '+' || d == '-') && (src[j - 1] == 'e' || src[j - 1] == 'E') &&
                    !(src.compare(k, 2, "0x") == 0 || src.compare(k, 2, "0X") == 0)) {
                    ++j;
                    continue;
                }
                break;
            }
            out->push_back({Token::Number, src.substr(k, j - k), k});
            k = j;
            continue;
        }
        if (c == '"' || c == '\'' || c == '#' || c == '\\' || c == '@' || c == '$' || c == '`')
            return fail(HIPMR_E_PARSE, std::string("expression: unsupported character '") + c +
                                           "' at " + std::to_string(k));
        bool matched = false;
        for (int p = 0; punct[p]; ++p) {
            size_t len = std::strlen(punct[p]);
            if (src.compare(k, len, punct[p]) == 0) {
                out->push_back({Token::Punct, punct[p], k});
                k += len;
                matched = true;
                break;
            }
        }
        if (!matched)
            return fail(HIPMR_E_PARSE, std::string("expression: unexpected character '") + c +
                                           "' at " + std::to_string(k));
    }
    out->push_back({Token::End, "", n});
    return HIPMR_OK;
}

// ---------------------------------------------------------------- classifier
namespace {

bool is_punct(const Token& t, const char* s) { return t.kind == Token::Punct && t.text == s; }

bool is_assign_op(const Token& t) {
    static const std::set<std::string> ops = {"=", "+=", "-=", "*=", "/=", "%=",
                                              "&=", "|=", "^=", "<<=", ">>="};
    return t.kind == Token::Punct && ops.count(t.text);
}

// name[i + E] / name[i - E] at toks[k]: E is built from literals, scalar
// arguments, n, + - * / % and parentheses (shifts and other operators only
// inside parentheses, so that i + (E) groups as written).  On a match,
// *close is the index of the closing ']' and *offset the signed distance.
bool match_shift(const std::vector<Token>& toks, size_t k, const Signature& sig, size_t* close,
                 std::string* offset) {
    if (!(k + 4 < toks.size() && is_punct(toks[k + 1], "[") && toks[k + 2].kind == Token::Ident &&
          toks[k + 2].text == "i" && (is_punct(toks[k + 3], "+") || is_punct(toks[k + 3], "-"))))
        return false;
    static const std::set<std::string> top = {"+", "-", "*", "/", "%", "(", ")"};
    static const std::set<std::string> nested = {"+", "-", "*", "/", "%", "(", ")", "<<", ">>", "&", "|", "^", "~"};
    int paren = 0;
    std::string text = "(0";
    bool operand = false;
    for (size_t j = k + 3; j < toks.size(); ++j) {
        const Token& t = toks[j];
        if (is_punct(t, "]") && paren == 0) {
            if (!operand) return false;
            *close = j;
            *offset = text + ")";
            return true;
        }
        if (t.kind == Token::Number) {
            operand = true;
        } else if (t.kind == Token::Ident) {
            bool scalar = t.text == "n";
            for (const ArgDecl& a : sig.args)
                if (a.name == t.text && !a.pointer) scalar = true;
            if (!scalar) return false;
            operand = true;
        } else if (t.kind == Token::Punct) {
            if (!(paren == 0 ? top : nested).count(t.text)) return false;
            if (t.text == "(") ++paren;
            if (t.text == ")" && --paren < 0) return false;
            operand = t.text == ")";
        } else {
            return false;
        }
        text += " " + t.text;
    }
    return false;
}

}  // namespace

hipmr_status classify(const std::vector<Token>& toks, Signature* sig, bool is_map, ExprInfo* out) {
    *out = ExprInfo();
    std::map<std::string, size_t> arg_index;
    for (size_t a = 0; a < sig->args.size(); ++a) {
        sig->args[a].read = sig->args[a].written = sig->args[a].write_only = false;
        sig->args[a].lane = sig->args[a].uniform = sig->args[a].shifted = sig->args[a].other = false;
        arg_index[sig->args[a].name] = a;
    }
    // balance of brackets; forbidden constructs
    std::vector<char> stack;
    bool saw_loop = false;
    for (const Token& t : toks) {
        if (t.kind == Token::Ident) {
            if (t.text == "return" || t.text == "goto" || t.text == "asm" || t.text == "__asm__" ||
                t.text == "__asm")
                return fail(HIPMR_E_UNSUPPORTED, "expression: '" + t.text + "' is not supported");
            if (t.text == "for" || t.text == "while" || t.text == "do" || t.text == "switch") saw_loop = true;
            if ((t.text == "break" || t.text == "continue") && !saw_loop)
                return fail(HIPMR_E_UNSUPPORTED, "expression: '" + t.text + "' outside a loop");
            if (has_reserved_prefix(t.text))
                return fail(HIPMR_E_PARSE, "expression: names starting with hipmr_ (any case) are reserved");
        }
        if (t.kind != Token::Punct) continue;
        char c = t.text[0];
        if (t.text.size() == 1 && (c == '(' || c == '[' || c == '{')) stack.push_back(c);
        if (t.text.size() == 1 && (c == ')' || c == ']' || c == '}')) {
            char want = c == ')' ? '(' : c == ']' ? '[' : '{';
            if (stack.empty() || stack.back() != want)
                return fail(HIPMR_E_PARSE, "expression: unbalanced '" + t.text + "' at " + std::to_string(t.pos));
            stack.pop_back();
        }
    }
    if (!stack.empty()) return fail(HIPMR_E_PARSE, "expression: unbalanced brackets");

    std::vector<bool> uncond_write(sig->args.size(), false);
    int depth = 0;   // ( and { nesting
    for (size_t k = 0; k + 1 < toks.size(); ++k) {
        const Token& t = toks[k];
        if (t.kind == Token::Punct) {
            if (t.text == "(" || t.text == "{" || t.text == "[") ++depth;
            if (t.text == ")" || t.text == "}" || t.text == "]") --depth;
            continue;
        }
        if (t.kind != Token::Ident) continue;
        if (k > 0 && (is_punct(toks[k - 1], ".") || is_punct(toks[k - 1], "->"))) continue;
        auto it = arg_index.find(t.text);
        if (it == arg_index.end()) continue;
        ArgDecl& a = sig->args[it->second];
        if (!a.pointer) {
            a.read = true;
            const Token& nx = toks[k + 1];
            bool pre = k > 0 && (is_punct(toks[k - 1], "++") || is_punct(toks[k - 1], "--"));
            if (is_assign_op(nx) || is_punct(nx, "++") || is_punct(nx, "--") || pre)
                return fail(HIPMR_E_UNSUPPORTED, "expression: the scalar argument '" + a.name +
                                                     "' may not be assigned");
            continue;
        }
        bool lane_local = k + 3 < toks.size() && is_punct(toks[k + 1], "[") &&
                          toks[k + 2].kind == Token::Ident && toks[k + 2].text == "i" &&
                          is_punct(toks[k + 3], "]");
        // a read of one fixed element (name[3]): uniform across i, read directly
        bool constant_index = !lane_local && k + 3 < toks.size() && is_punct(toks[k + 1], "[") &&
                              toks[k + 2].kind == Token::Number && is_punct(toks[k + 3], "]");
        // a read at a uniform distance from i
        size_t close = 0;
        std::string offset;
        bool shifted = !lane_local && !constant_index && match_shift(toks, k, *sig, &close, &offset);
        size_t after;   // token after the closing ']'
        if (lane_local) {
            after = k + 4;
            a.lane = true;
        } else if (constant_index) {
            after = k + 4;
            a.uniform = true;
        } else if (shifted) {
            after = close + 1;
            a.shifted = true;
            bool known = false;
            for (const ShiftRead& r : out->shifts) known |= r.arg == it->second && r.offset == offset;
            if (!known) out->shifts.push_back(ShiftRead{it->second, offset});
        } else {
            out->vectorizable = false;
            a.other = true;
            if (!(k + 1 < toks.size() && is_punct(toks[k + 1], "["))) {
                // bare array name (pointer arithmetic etc.): treat as read and write
                a.read = true;
                if (!a.is_const) a.written = true;
                continue;
            }
            int d = 0;
            size_t j = k + 1;
            for (; j < toks.size(); ++j) {
                if (is_punct(toks[j], "[")) ++d;
                if (is_punct(toks[j], "]") && --d == 0) break;
            }
            after = j + 1;
        }
        const Token& nx = toks[after < toks.size() ? after : toks.size() - 1];
        bool pre = k > 0 && (is_punct(toks[k - 1], "++") || is_punct(toks[k - 1], "--"));
        bool incdec = pre || is_punct(nx, "++") || is_punct(nx, "--");
        if (incdec || (is_assign_op(nx) && nx.text != "=")) {
            a.read = a.written = true;
        } else if (is_punct(nx, "=")) {
            a.written = true;
            bool stmt_start = k == 0 || is_punct(toks[k - 1], ";") || is_punct(toks[k - 1], "}");
            if (lane_local && stmt_start && depth == 0) uncond_write[it->second] = true;
        } else {
            a.read = true;
        }
        if (a.written && a.is_const)
            return fail(HIPMR_E_PARSE, "expression: assignment to const array '" + a.name + "'");
    }
    for (size_t a = 0; a < sig->args.size(); ++a) {
        ArgDecl& d = sig->args[a];
        d.write_only = d.pointer && d.written && !d.read && uncond_write[a];
        if (d.written) out->has_writes = true;
        // a fixed element of an array the expression also writes could be
        // written by another i: keep such expressions on the one-element path
        if (d.uniform && d.written) out->vectorizable = false;
        // so could a shifted element
        if (d.shifted && d.written) out->vectorizable = false;
    }
    if (!out->vectorizable) out->shifts.clear();
    if (is_map && out->has_writes)
        return fail(HIPMR_E_UNSUPPORTED, "expression: a map expression may not assign to arrays");
    return HIPMR_OK;
}

std::string vectorize_accesses(const std::vector<Token>& toks, const Signature& sig,
                               const std::vector<ShiftRead>& shifts) {
    std::set<std::string> arrays;
    for (auto& a : sig.args)
        if (a.pointer) arrays.insert(a.name);
    std::string s;
    for (size_t k = 0; k < toks.size() && toks[k].kind != Token::End; ++k) {
        const Token& t = toks[k];
        size_t close = 0;
        std::string offset;
        if (!shifts.empty() && t.kind == Token::Ident && arrays.count(t.text) &&
            !(k > 0 && (is_punct(toks[k - 1], ".") || is_punct(toks[k - 1], "->"))) &&
            match_shift(toks, k, sig, &close, &offset)) {
            for (size_t r = 0; r < shifts.size(); ++r)
                if (sig.args[shifts[r].arg].name == t.text && shifts[r].offset == offset) {
                    s += " hipmr_q" + std::to_string(r) + "[hipmr_u].v[hipmr_j]";
                    k = close;
                    break;
                }
            if (k == close) continue;
        }
        if (t.kind == Token::Ident && arrays.count(t.text) && k + 3 < toks.size() &&
            is_punct(toks[k + 1], "[") && toks[k + 2].kind == Token::Ident && toks[k + 2].text == "i" &&
            is_punct(toks[k + 3], "]") &&
            !(k > 0 && (is_punct(toks[k - 1], ".") || is_punct(toks[k - 1], "->")))) {
            s += " hipmr_p_" + t.text + "[hipmr_u].v[hipmr_j]";
            k += 3;
            continue;
        }
        s += ' ';
        s += t.text;
    }
    return s;
}

std::string join_tokens(const std::vector<Token>& toks) {
    std::string s;
    for (auto& t : toks) {
        if (t.kind == Token::End) break;
        s += ' ';
        s += t.text;
    }
    return s;
}

Combine canonical_combine(const std::string& combine) {
    std::string s;
    for (char c : combine)
        if (!std::isspace((unsigned char)c)) s += c;
    if (s == "a+b" || s == "b+a" || s == "sum") return Combine::Sum;
    if (s == "max(a,b)" || s == "max(b,a)" || s == "max") return Combine::Max;
    if (s == "min(a,b)" || s == "min(b,a)" || s == "min") return Combine::Min;
    return Combine::Generic;
}

}  // namespace hipmr
