"""Tokenizer for the C subset in which users write elementwise statements,
map expressions, combine expressions and neutral elements.

Oracle (test infrastructure): the kernels are given as C source text
(section "Core Method", kernels-as-strings; section "Efficient Evaluation of
Element-wise Expressions" for the statement list over the formal index ``i``;
section "Map-Reduce" for the map / reduce expressions and the neutral
element).  This module shares no code with the GPU library.
"""

from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

PUNCT = sorted(
    """<<= >>= ++ -- << >> <= >= == != && || += -= *= /= %= &= |= ^=
       + - * / % < > = ! ~ & | ^ ? : , ; ( ) [ ] { }""".split(),
    key=len, reverse=True)


class CSyntaxError(ValueError):
    """Raised for text outside the supported C subset."""


@dataclass(frozen=True)
class Tok:
    kind: str      # 'id', 'int', 'float', 'op', 'end'
    text: str
    pos: int
    value: object = None   # int value or Fraction for numbers
    suffix: str = ""


def _int_literal(text, pos):
    body = text
    suffix = ""
    while body and body[-1] in "uUlL":
        suffix = body[-1].lower() + suffix
        body = body[:-1]
    if body.lower().startswith("0x"):
        value, radix = int(body[2:], 16), 16
    elif len(body) > 1 and body.startswith("0"):
        value, radix = int(body[1:], 8), 8
    else:
        value, radix = int(body, 10), 10
    if suffix not in ("", "u", "l", "ll", "ul", "ull", "lu", "llu"):
        raise CSyntaxError(f"bad integer suffix in {text!r} at {pos}")
    return Tok("int", text, pos, value, suffix + ("#dec" if radix == 10 else "#nondec"))


def _float_literal(text, pos):
    body, suffix = text, ""
    if body[-1] in "fFlL":
        suffix, body = body[-1].lower(), body[:-1]
    try:
        value = Fraction(body)
    except ValueError as exc:
        raise CSyntaxError(f"bad floating literal {text!r} at {pos}") from exc
    return Tok("float", text, pos, value, suffix)


def tokenize(src: str) -> list[Tok]:
    toks: list[Tok] = []
    k, n = 0, len(src)
    while k < n:
        c = src[k]
        if c.isspace():
            k += 1
            continue
        if src.startswith("//", k):
            j = src.find("\n", k)
            k = n if j < 0 else j + 1
            continue
        if src.startswith("/*", k):
            j = src.find("*/", k + 2)
            if j < 0:
                raise CSyntaxError("unterminated comment")
            k = j + 2
            continue
        if c.isalpha() or c == "_":
            j = k + 1
            while j < n and (src[j].isalnum() or src[j] == "_"):
                j += 1
            toks.append(Tok("id", src[k:j], k))
            k = j
            continue
        if c.isdigit() or (c == "." and k + 1 < n and src[k + 1].isdigit()):
            j = k
            if src.startswith(("0x", "0X"), k):
                j = k + 2
                while j < n and (src[j] in "0123456789abcdefABCDEF"):
                    j += 1
                while j < n and src[j] in "uUlL":
                    j += 1
                toks.append(_int_literal(src[k:j], k))
                k = j
                continue
            is_float = False
            while j < n and src[j].isdigit():
                j += 1
            if j < n and src[j] == ".":
                is_float = True
                j += 1
                while j < n and src[j].isdigit():
                    j += 1
            if j < n and src[j] in "eE":
                m = j + 1
                if m < n and src[m] in "+-":
                    m += 1
                if m < n and src[m].isdigit():
                    is_float = True
                    j = m
                    while j < n and src[j].isdigit():
                        j += 1
            if is_float:
                if j < n and src[j] in "fFlL":
                    j += 1
                toks.append(_float_literal(src[k:j], k))
            else:
                while j < n and src[j] in "uUlL":
                    j += 1
                toks.append(_int_literal(src[k:j], k))
            if j < n and (src[j].isalnum() or src[j] == "_"):
                raise CSyntaxError(f"bad number at {k}: {src[k:j + 1]!r}")
            k = j
            continue
        for p in PUNCT:
            if src.startswith(p, k):
                toks.append(Tok("op", p, k))
                k += len(p)
                break
        else:
            raise CSyntaxError(f"unexpected character {c!r} at {k}")
    toks.append(Tok("end", "", n))
    return toks
