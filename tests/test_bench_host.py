"""Host-side piece of bench.py: the source identity that keys the stored
traffic counters (the one-GPU refusal is tested with the C-ABI host tests)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_text_drops_comments_and_keeps_literals():
    src = ('#include <x.h>   // a header\n'
           '\n'
           '/* block\n   comment */ int a = 1; // trailing\n'
           'const char *s = "not // a comment /* either */";\n'
           "char c = '/';  char q = '\\'';\n"
           'const char *e = "esc \\" // still inside";\n')
    out = bench.code_text(src)
    assert out.splitlines() == [
        '#include <x.h>',
        'int a = 1;',
        'const char *s = "not // a comment /* either */";',
        "char c = '/'; char q = '\\'';",
        'const char *e = "esc \\" // still inside";',
    ]


def test_code_text_ignores_comment_and_spacing_edits_only():
    a = "int f(int x)\n{\n    return x + 1;   // one more\n}\n"
    b = "// increment\nint f(int x)\n{\n\n  return x + 1;\n}\n"
    c = "int f(int x)\n{\n    return x + 2;\n}\n"
    assert bench.code_text(a) == bench.code_text(b)
    assert bench.code_text(a) != bench.code_text(c)


def test_kernel_hash_matches_stored_traffic_key_format():
    h = bench.kernel_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    with open(bench.TRAFFIC_FILE) as f:
        stored = json.load(f)
    assert len(stored["kernel_hash"]) == 16

