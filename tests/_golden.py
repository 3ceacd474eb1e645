import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def kv(name: str) -> dict:
    """key = value lines; '#' starts a comment; values stay strings."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = line.split("=", 1)
            out[k.strip()] = v.strip()
    return out


def table(name: str) -> list:
    """Whitespace-separated rows; the last comment line before data names the columns."""
    header, rows = None, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            s = line.strip()
            if not s:
                continue
            if s.startswith("#"):
                header = s[1:].split()
                continue
            rows.append(dict(zip(header, s.split())))
    return rows
