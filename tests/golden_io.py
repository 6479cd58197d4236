"""Reader for ``tests/golden/hand_examples.txt`` (hand-derived expectations)."""

from __future__ import annotations

import dataclasses
from pathlib import Path

GOLDEN = Path(__file__).resolve().parent / "golden" / "hand_examples.txt"


@dataclasses.dataclass
class Example:
    name: str
    cite: str
    patterns: list[bytes]
    text: bytes
    matches: list[tuple[int, int]]
    counts: list[int]


def _hex_list(s: str) -> list[bytes]:
    return [] if s.strip() == "-" else [bytes.fromhex(h) for h in s.split()]


def load_examples(path: Path = GOLDEN) -> list[Example]:
    blocks: list[dict] = []
    cur: dict = {}
    for raw in path.read_text().splitlines():
        line = raw.strip()
        if not line or line.startswith("#"):
            continue
        key, _, val = line.partition(":")
        key, val = key.strip(), val.strip()
        if key == "name":
            if cur:
                blocks.append(cur)
            cur = {}
        cur[key] = val
    if cur:
        blocks.append(cur)
    out = []
    for b in blocks:
        text = b"" if b["text"] == "-" else bytes.fromhex(b["text"])
        matches = []
        if b["matches"] != "-":
            for tok in b["matches"].split():
                o, j = tok.split(":")
                matches.append((int(o), int(j)))
        out.append(Example(b["name"], b["cite"], _hex_list(b["patterns"]), text, matches,
                           [int(c) for c in b["counts"].split()]))
    return out
