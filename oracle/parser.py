"""Recursive-descent parser for the C statement / expression subset.

Oracle (test infrastructure).  The paper passes device code as C source
strings (section "Core Method"); an elementwise operation is "a statement
(or semicolon-separated list of statements)" executed for each value of the
formal index ``i`` (section "Efficient Evaluation of Element-wise
Expressions"), and a reduction takes a map expression, a reduce expression
in the formal arguments ``a`` and ``b``, and a neutral-element expression
(section "Map-Reduce").  This module turns that text into a small AST with
the usual C operator precedence; evaluation lives in ``interp``.
"""

from __future__ import annotations

from dataclasses import dataclass, field

from .lexer import CSyntaxError, Tok, tokenize

# C type spellings accepted in casts and local declarations, mapped to the
# oracle's storage type names (see ``ctype.STORAGE_VT``).
TYPE_WORDS = {
    ("float",): "float32", ("double",): "float64",
    ("int",): "int32", ("signed",): "int32", ("signed", "int"): "int32",
    ("int32_t",): "int32",
    ("unsigned",): "uint32", ("unsigned", "int"): "uint32", ("uint32_t",): "uint32",
    ("long",): "int64", ("long", "int"): "int64", ("long", "long"): "int64",
    ("long", "long", "int"): "int64", ("int64_t",): "int64",
    ("short",): "int16", ("short", "int"): "int16", ("int16_t",): "int16",
    ("unsigned", "short"): "uint16", ("uint16_t",): "uint16",
    ("char",): "int8", ("signed", "char"): "int8", ("int8_t",): "int8",
    ("unsigned", "char"): "uint8", ("uint8_t",): "uint8",
    ("bool",): "bool",
    ("bfloat16",): "bfloat16", ("__hip_bfloat16",): "bfloat16",
    ("half",): "float16", ("__half",): "float16", ("_Float16",): "float16",
    ("float16",): "float16",
    ("fp8_e4m3",): "fp8_e4m3",
    ("complex64",): "complex64", ("cfloat",): "complex64",
}
_TYPE_FIRST = {w[0] for w in TYPE_WORDS}


# ----------------------------------------------------------------- AST nodes
@dataclass
class Num:
    value: object          # int or Fraction
    is_float: bool
    suffix: str


@dataclass
class Name:
    ident: str


@dataclass
class Index:
    base: str
    index: object


@dataclass
class Call:
    func: str
    args: list


@dataclass
class Unary:
    op: str
    operand: object


@dataclass
class Binary:
    op: str
    left: object
    right: object


@dataclass
class Logical:
    op: str                # '&&' or '||'
    left: object
    right: object


@dataclass
class Cond:
    cond: object
    then: object
    other: object


@dataclass
class Cast:
    type: str
    operand: object


@dataclass
class Assign:
    op: str                # '=', '+=', ...
    target: object         # Name or Index
    value: object


@dataclass
class IncDec:
    op: str                # '++' or '--'
    target: object
    prefix: bool


@dataclass
class Comma:
    left: object
    right: object


@dataclass
class ExprStmt:
    expr: object


@dataclass
class Decl:
    type: str
    items: list = field(default_factory=list)   # [(name, init-or-None)]


@dataclass
class If:
    cond: object
    then: object
    other: object = None


@dataclass
class Block:
    stmts: list


ASSIGN_OPS = ("=", "+=", "-=", "*=", "/=", "%=", "&=", "|=", "^=", "<<=", ">>=")
BINARY_LEVELS = [
    ("|",), ("^",), ("&",), ("==", "!="), ("<", ">", "<=", ">="),
    ("<<", ">>"), ("+", "-"), ("*", "/", "%"),
]


class _Parser:
    def __init__(self, src: str):
        self.toks: list[Tok] = tokenize(src)
        self.k = 0

    # -- helpers
    def peek(self, off=0) -> Tok:
        return self.toks[min(self.k + off, len(self.toks) - 1)]

    def next(self) -> Tok:
        t = self.toks[self.k]
        self.k += 1
        return t

    def accept(self, text) -> bool:
        t = self.peek()
        if t.kind in ("op", "id") and t.text == text:
            self.k += 1
            return True
        return False

    def expect(self, text):
        if not self.accept(text):
            t = self.peek()
            raise CSyntaxError(f"expected {text!r} at {t.pos}, found {t.text!r}")

    def _type_at(self, off=0):
        """Longest type-name match starting at token offset; returns (type, ntok)."""
        words = []
        j = off
        if self.peek(j).kind == "id" and self.peek(j).text == "const":
            j += 1
        start = j
        best = None
        while self.peek(j).kind == "id":
            words.append(self.peek(j).text)
            j += 1
            if tuple(words) in TYPE_WORDS:
                best = (TYPE_WORDS[tuple(words)], j - off)
            if len(words) >= 3:
                break
        if best is None or self.peek(start).text not in _TYPE_FIRST:
            return None
        return best

    # -- statements
    def statements(self, closing=None):
        stmts = []
        while True:
            t = self.peek()
            if t.kind == "end" or (closing and t.kind == "op" and t.text == closing):
                return stmts
            if self.accept(";"):
                continue
            stmts.append(self.statement())

    def statement(self):
        if self.accept("{"):
            body = self.statements(closing="}")
            self.expect("}")
            return Block(body)
        if self.peek().kind == "id" and self.peek().text == "if":
            self.next()
            self.expect("(")
            cond = self.expression()
            self.expect(")")
            then = self.statement()
            other = None
            if self.peek().kind == "id" and self.peek().text == "else":
                self.next()
                other = self.statement()
            return If(cond, then, other)
        if self.peek().kind == "id" and self.peek().text in (
                "for", "while", "do", "switch", "return", "goto", "break", "continue"):
            raise CSyntaxError(f"unsupported statement {self.peek().text!r}")
        ty = self._type_at()
        if ty is not None and self.peek(ty[1]).kind == "id":
            self.k += ty[1]
            decl = Decl(ty[0])
            while True:
                name = self.next()
                if name.kind != "id":
                    raise CSyntaxError(f"expected a name at {name.pos}")
                init = None
                if self.accept("="):
                    init = self.assignment()
                decl.items.append((name.text, init))
                if not self.accept(","):
                    break
            self._end_statement()
            return decl
        e = self.expression()
        self._end_statement()
        return ExprStmt(e)

    def _end_statement(self):
        t = self.peek()
        if t.kind == "end" or (t.kind == "op" and t.text == "}"):
            return
        self.expect(";")

    # -- expressions
    def expression(self):
        e = self.assignment()
        while self.accept(","):
            e = Comma(e, self.assignment())
        return e

    def assignment(self):
        start = self.k
        lhs = self.conditional()
        t = self.peek()
        if t.kind == "op" and t.text in ASSIGN_OPS:
            if not isinstance(lhs, (Name, Index)):
                raise CSyntaxError(f"assignment to a non-lvalue at {self.toks[start].pos}")
            self.next()
            return Assign(t.text, lhs, self.assignment())
        return lhs

    def conditional(self):
        c = self.logical_or()
        if self.accept("?"):
            a = self.expression()
            self.expect(":")
            b = self.conditional()
            return Cond(c, a, b)
        return c

    def logical_or(self):
        e = self.logical_and()
        while self.accept("||"):
            e = Logical("||", e, self.logical_and())
        return e

    def logical_and(self):
        e = self.binary(0)
        while self.accept("&&"):
            e = Logical("&&", e, self.binary(0))
        return e

    def binary(self, level):
        if level == len(BINARY_LEVELS):
            return self.cast()
        e = self.binary(level + 1)
        while True:
            t = self.peek()
            if t.kind == "op" and t.text in BINARY_LEVELS[level]:
                self.next()
                e = Binary(t.text, e, self.binary(level + 1))
            else:
                return e

    def cast(self):
        if self.peek().kind == "op" and self.peek().text == "(":
            ty = self._type_at(1)
            if ty is not None and self.peek(1 + ty[1]).text == ")":
                self.k += 1 + ty[1] + 1
                return Cast(ty[0], self.cast())
        return self.unary()

    def unary(self):
        t = self.peek()
        if t.kind == "op" and t.text in ("+", "-", "!", "~"):
            self.next()
            return Unary(t.text, self.cast())
        if t.kind == "op" and t.text in ("++", "--"):
            self.next()
            target = self.unary()
            if not isinstance(target, (Name, Index)):
                raise CSyntaxError("increment of a non-lvalue")
            return IncDec(t.text, target, True)
        return self.postfix()

    def postfix(self):
        e = self.primary()
        while True:
            t = self.peek()
            if t.kind == "op" and t.text == "[":
                if not isinstance(e, Name):
                    raise CSyntaxError(f"subscript of a non-array at {t.pos}")
                self.next()
                idx = self.expression()
                self.expect("]")
                e = Index(e.ident, idx)
            elif t.kind == "op" and t.text in ("++", "--"):
                if not isinstance(e, (Name, Index)):
                    raise CSyntaxError("increment of a non-lvalue")
                self.next()
                e = IncDec(t.text, e, False)
            else:
                return e

    def primary(self):
        t = self.next()
        if t.kind == "int":
            return Num(t.value, False, t.suffix)
        if t.kind == "float":
            return Num(t.value, True, t.suffix)
        if t.kind == "op" and t.text == "(":
            e = self.expression()
            self.expect(")")
            return e
        if t.kind == "id":
            # functional cast, e.g. float(k[i])
            self.k -= 1
            ty = self._type_at()
            if ty is not None and self.peek(ty[1]).text == "(":
                self.k += ty[1] + 1
                e = self.expression()
                self.expect(")")
                return Cast(ty[0], e)
            self.k += 1
            if self.peek().kind == "op" and self.peek().text == "(":
                self.next()
                args = []
                if not self.accept(")"):
                    while True:
                        args.append(self.assignment())
                        if self.accept(")"):
                            break
                        self.expect(",")
                return Call(t.text, args)
            return Name(t.text)
        raise CSyntaxError(f"unexpected {t.text!r} at {t.pos}")


def parse_statements(src: str) -> list:
    p = _Parser(src)
    stmts = p.statements()
    if p.peek().kind != "end":
        raise CSyntaxError(f"trailing text at {p.peek().pos}")
    return stmts


def parse_expression(src: str):
    p = _Parser(src)
    e = p.expression()
    if p.peek().kind != "end":
        raise CSyntaxError(f"trailing text at {p.peek().pos}: {p.peek().text!r}")
    return e
