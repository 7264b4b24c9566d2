"""Bindings of the extension entry points of libstt (filled in as they are exported)."""
from __future__ import annotations


def bind(L) -> None:
    return None
