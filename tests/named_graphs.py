"""Named test graphs by the names used in tests/golden/closed_forms.json."""
import re

import graphgen as gg


def by_name(name: str):
    m = re.fullmatch(r"K(\d+)", name)
    if m:
        return gg.complete(int(m.group(1)))
    m = re.fullmatch(r"K(\d+),(\d+)", name)
    if m:
        return gg.complete_bipartite(int(m.group(1)), int(m.group(2)))
    m = re.fullmatch(r"C(\d+)", name)
    if m:
        return gg.cycle(int(m.group(1)))
    m = re.fullmatch(r"grid(\d+)x(\d+)", name)
    if m:
        return gg.grid(int(m.group(1)), int(m.group(2)))
    m = re.fullmatch(r"Q(\d+)", name)
    if m:
        return gg.hypercube(int(m.group(1)))
    m = re.fullmatch(r"S(\d+)", name)
    if m:
        return gg.star(int(m.group(1)))
    if name == "petersen":
        return gg.petersen()
    raise KeyError(name)
